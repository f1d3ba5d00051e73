// Online autotuner of launch shapes: see tune.h.
#include "tune.h"

#include <algorithm>
#include <array>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace hpt {
namespace {

struct Pending {
  int cand;
  hipEvent_t e0, e1;
};

struct ClassState {
  int ncand = 0;
  int calls = 0;
  int choice = -1;                       // decided variant, -1 while tuning
  std::vector<std::vector<float>> ms;    // completed measurements per variant
  std::vector<Pending> pending;          // launched, not yet read
};

using Key = std::array<int64_t, 4>;

std::mutex g_mu;
bool g_on = true;
std::map<Key, ClassState> g_classes;
uint64_t g_picks = 0;
constexpr size_t MAX_CLASSES = 1 << 16;   // past this, new shape classes run the default untimed

const char* site_name(int site) {
  switch (site) {
    case TUNE_MODE_STRIPS: return "mode_product_strips";
    case TUNE_MODE_LEAD: return "mode_product_lead";
    case TUNE_PERMUTE_LEAD: return "permute_first_leg";
    default: return "?";
  }
}

// read the pending measurements that have completed (never blocks)
void poll(ClassState& st) {
  std::vector<Pending> keep;
  for (const Pending& p : st.pending) {
    if (hipEventQuery(p.e1) == hipSuccess) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, p.e0, p.e1) == hipSuccess && p.cand < st.ncand) st.ms[p.cand].push_back(t);
      (void)hipEventDestroy(p.e0);
      (void)hipEventDestroy(p.e1);
    } else {
      keep.push_back(p);
    }
  }
  st.pending.swap(keep);
  if (st.choice >= 0 || st.ncand <= 0) return;
  for (int c = 0; c < st.ncand; ++c)
    if ((int)st.ms[c].size() < TUNE_REPS) return;
  int best = 0;
  float bt = *std::min_element(st.ms[0].begin(), st.ms[0].end());
  for (int c = 1; c < st.ncand; ++c) {
    const float t = *std::min_element(st.ms[c].begin(), st.ms[c].end());
    if (t < bt) {
      bt = t;
      best = c;
    }
  }
  st.choice = best;
}

}  // namespace

int tune_pick(int site, int64_t k0, int64_t k1, int64_t k2, int ncand, TuneCall* c) {
  c->site = site;
  c->key[0] = k0;
  c->key[1] = k1;
  c->key[2] = k2;
  c->timed = false;
  c->cand = 0;
  if (ncand <= 1) return 0;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_on) return 0;
  // every 1024 picks, read the finished measurements of every class, so the
  // events of classes that are not called again are released
  if ((++g_picks & 1023) == 0)
    for (auto& kv : g_classes)
      if (!kv.second.pending.empty()) poll(kv.second);
  const Key key{site, k0, k1, k2};
  auto it = g_classes.find(key);
  if (it == g_classes.end() && g_classes.size() >= MAX_CLASSES) return 0;
  ClassState& st = it != g_classes.end() ? it->second : g_classes[key];
  if (st.ncand != ncand) {
    st = ClassState();
    st.ncand = ncand;
    st.ms.assign(ncand, {});
  }
  poll(st);
  if (st.choice >= 0) {
    c->cand = st.choice;
    return c->cand;
  }
  // still tuning: the next variant in turn, timed (bounded: a class whose
  // events never complete stops being timed and keeps the default)
  if (st.pending.size() >= 64) return 0;
  c->cand = st.calls % ncand;
  ++st.calls;
  c->timed = true;
  return c->cand;
}

void tune_begin(TuneCall* c, hipStream_t s) {
  if (!c->timed) return;
  if (hipEventCreate(&c->e0) != hipSuccess || hipEventCreate(&c->e1) != hipSuccess ||
      hipEventRecord(c->e0, s) != hipSuccess) {
    if (c->e0) (void)hipEventDestroy(c->e0);
    if (c->e1) (void)hipEventDestroy(c->e1);
    c->e0 = c->e1 = nullptr;
    c->timed = false;
  }
}

void tune_end(TuneCall* c, hipStream_t s) {
  if (!c->timed) return;
  if (hipEventRecord(c->e1, s) != hipSuccess) {
    (void)hipEventDestroy(c->e0);
    (void)hipEventDestroy(c->e1);
    c->timed = false;
    return;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  ClassState& st = g_classes[Key{c->site, c->key[0], c->key[1], c->key[2]}];
  st.pending.push_back(Pending{c->cand, c->e0, c->e1});
  c->timed = false;
}

int tune_set(int mode) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (mode == 0 || mode == 1) {
    g_on = mode == 1;
    return 0;
  }
  if (mode == 2) {
    for (auto& kv : g_classes)
      for (const Pending& p : kv.second.pending) {
        (void)hipEventSynchronize(p.e1);
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
      }
    g_classes.clear();
    return 0;
  }
  return -1;
}

int tune_report(char* buf, uint64_t cap, uint64_t* needed) {
  std::string out;
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& kv : g_classes) {
    ClassState& st = kv.second;
    poll(st);
    char line[512];
    int n = snprintf(line, sizeof(line), "%s %lld %lld %lld:", site_name((int)kv.first[0]), (long long)kv.first[1],
                     (long long)kv.first[2], (long long)kv.first[3]);
    out.append(line, (size_t)std::max(n, 0));
    for (int c = 0; c < st.ncand; ++c) {
      if (st.ms[c].empty())
        n = snprintf(line, sizeof(line), " -");
      else
        n = snprintf(line, sizeof(line), " %.4f", (double)*std::min_element(st.ms[c].begin(), st.ms[c].end()));
      out.append(line, (size_t)std::max(n, 0));
    }
    n = snprintf(line, sizeof(line), " -> %d\n", st.choice);
    out.append(line, (size_t)std::max(n, 0));
  }
  if (needed) *needed = out.size() + 1;
  if (buf && cap > 0) {
    const size_t k = std::min<size_t>(out.size(), (size_t)cap - 1);
    std::copy(out.begin(), out.begin() + k, buf);
    buf[k] = 0;
  }
  return 0;
}

}  // namespace hpt
