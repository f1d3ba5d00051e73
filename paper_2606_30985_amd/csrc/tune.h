// Online autotuner of launch shapes (tune.hip).
//
// A tunable launch site offers several variants that compute every output
// with the same operations in the same order (different strip heights, grid
// sizes or transpose tilings of the same arithmetic), so the choice changes
// the time and never a result.  For each shape class the first calls run the
// candidates in turn, each bracketed by two HIP events on the launch stream;
// the elapsed times are read later without blocking (hipEventQuery at the
// next call of the same class), and once every candidate has TUNE_REPS
// measurements the fastest (minimum over its repeats, lowest index on a tie)
// is used from then on.  With tuning off every site runs candidate 0, the
// untuned default.
#pragma once
#include <cstdint>

#include "common.h"

namespace hpt {

enum TuneSite : int {
  TUNE_MODE_STRIPS = 0,   // mode product, even inner >= 32: strip height and grid
  TUNE_MODE_LEAD = 1,     // mode product on the leading leg: grid
  TUNE_PERMUTE_LEAD = 2,  // cut leg moved from / to the first position: tile or panel transpose
  TUNE_SITES
};

constexpr int TUNE_REPS = 2;

struct TuneCall {
  int site = -1;
  int64_t key[3] = {0, 0, 0};
  int cand = 0;
  bool timed = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

// The variant to launch (0 <= result < ncand) for this call of `site` with
// shape class key; fills c.  When c->timed is set the caller wraps exactly
// its launches of the variant in tune_begin / tune_end on stream s.
int tune_pick(int site, int64_t k0, int64_t k1, int64_t k2, int ncand, TuneCall* c);
void tune_begin(TuneCall* c, hipStream_t s);
void tune_end(TuneCall* c, hipStream_t s);

// 1: on (the default), 0: off (candidate 0 everywhere); 2: forget every
// decision and measurement (tuning stays as it was)
int tune_set(int mode);
// one line per shape class: site, key, per-candidate best milliseconds, choice
int tune_report(char* buf, uint64_t cap, uint64_t* needed);

}  // namespace hpt
