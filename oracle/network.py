"""The method, step by step, in FP64 NumPy (oracle; test infrastructure only).

Paper sections followed (cited by section / equation / algorithm name):

* Sec. "Pauli Basis Tensor Network": the operator Z_c(t) is a network of
  real site tensors psi_v[i_1..i_deg, p], Pauli leg p in (I, X, Y, Z), live
  bond dimension growing from 1; at t = 0 psi_c = e_Z, all other psi_v = e_I.
* Sec. "Trotter Decomposition", Eq. trotter: field half-step, 4-colour sweep
  of two-site gates, field half-step.
* Sec. "Gate Update" and Algorithm "Gate update for bond (v1, v2)":
  environment absorption with sqrt(mu), permutation of the cut leg next to the
  Pauli leg, QR, bond matrix over the cut (the k1 D x k2 D bond matrix of the
  implementation pipeline figure), gate on the Pauli pair, SVD and
  truncation (Eq. truncation), reconstruction Q M, inverse permutation,
  deabsorption, mu <- diag(lambda) with Vidal normalisation (Eq. vidal_norm).
* Sec. "BP Message Update", Eq. bp, Eq. bp_tol and Eq. damping: gauge BP.
* Sec. "Correlation Function via Belief Propagation", Eqs. bethe_raw, ze and
  bethe: measurement BP on the pinned network and the log-space Bethe sum
  with explicit signs.
* Table "Runtime diagnostic measures": gate_err, Bethe norm, sweeps/delta,
  S_e / log chi.

Readings of points the paper leaves open:
* Bond matrix contracts R_1, R_2 over the cut bond; the SVD acts on the
  (k1*4) x (k2*4) matrix.
* Gauge BP runs on the norm network sum_p psi psi with chi x chi symmetric
  messages, synchronous sweeps, Frobenius normalisation, damping
  M <- normalise((1-a) M + a normalise(sym(M_hat))), delta = max |change|.
* Measurement BP runs on the pinned single-layer network with vector
  messages, L2 normalisation and sign continuity.
* Tensors keep raw sqrt(s) (M_1 = U sqrt(S), M_2 = V sqrt(S)); only messages
  carry the normalised lambda; ||s|| in lambda is over the kept values.
* pseudo_sqrt drops eigenvalues w <= eps_pinv * w_max.
* Sign gauge: after the SVD, channel j is flipped (u_j, v_j -> -u_j, -v_j)
  when <w, cv1_new[:, j, :]> < 0, with w a SplitMix64-derived weight over
  site v1's flat (env, p) index.
"""

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .lattice import Lattice
from .ptm import field_ptm, coupling_ptm

# measurement flags (same bit meaning as the C library; values are an interface)
FLAG_BP_NOT_CONVERGED_GAUGE = 1 << 0
FLAG_BP_NOT_CONVERGED_MEAS = 1 << 1
FLAG_TRAP_CANDIDATE = 1 << 2
FLAG_NORM_EXPLODED = 1 << 3
FLAG_DEGENERATE_CUT = 1 << 4
FLAG_PINV_CUT = 1 << 5
FLAG_BETHE_ZERO = 1 << 6
FLAG_QR_FALLBACK = 1 << 7
FLAG_QR_RANK_DEFICIENT = 1 << 8
FLAG_TRAP_REMEDIATED = 1 << 9
FLAG_TRAP_UNRESOLVED = 1 << 10


@dataclass
class Config:
    Lx: int = 3
    Ly: int = 3
    J: float = 1.0
    h: float = 1.0
    dt: float = 0.05
    chi_max: int = 8
    centre: Optional[int] = None          # site id; None -> lattice centre
    eps_cut: float = 1e-11
    eps_pinv: float = 1e-12
    bp_alpha: float = 0.5
    bp_tol: float = 1e-10
    bp_max_sweeps: int = 1000
    bp_init: str = "uniform"             # "uniform" | "warm"
    meas_alpha: Optional[float] = None    # None -> bp_alpha
    meas_tol: Optional[float] = None      # None -> bp_tol
    meas_max_sweeps: Optional[int] = None
    gauge_bp: bool = True
    trap_sweeps: int = 30                 # trap-candidate threshold (sweeps)
    trap_retry: bool = False              # remediate verified traps (run.remediate_trap)
    trap_alpha: Optional[float] = None    # damping of the retry; None -> paper's rule
    model_axes: str = "paper"             # "paper": H = -J sum XX - h sum Z, observable Z_c (Eq.
                                          # hamiltonian); "zzx": H = -J sum ZZ - h sum X, observable Z_c


# --------------------------------------------------------------------------
# small helpers

def mode_product(T, S, axis):
    """out[.., a, ..] = sum_b S[a, b] T[.., b, ..] on the given axis."""
    out = np.tensordot(S, T, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def pseudo_sqrt(M, eps_pinv):
    """sqrt(M) and its pseudo-inverse for a symmetric PSD message.

    Paper, Algorithm "Gate update", first step (symmetrise, eigendecompose,
    form sqrt(mu) and mu^{-1/2}).  Eigenvalues w <= eps_pinv * max(w) (and
    negative rounding noise) are dropped from both.
    """
    Ms = 0.5 * (M + M.T)
    w, V = np.linalg.eigh(Ms)
    wmax = max(float(w.max()), 0.0)
    if wmax <= 0.0:
        raise FloatingPointError("environment message is zero")
    keep = w > eps_pinv * wmax
    sq = np.where(keep, np.sqrt(np.where(keep, w, 1.0)), 0.0)
    isq = np.where(keep, 1.0 / np.sqrt(np.where(keep, w, 1.0)), 0.0)
    S = (V * sq[None, :]) @ V.T
    Sinv = (V * isq[None, :]) @ V.T
    return S, Sinv, int(np.count_nonzero(~keep))


_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(n):
    """The first n outputs of SplitMix64 started from state 0, as uint64.

    SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
    generators", OOPSLA 2014): state_i = (i + 1) * gamma, then the finaliser
    z ^= z >> 30; z *= c1; z ^= z >> 27; z *= c2; z ^= z >> 31.
    """
    with np.errstate(over="ignore"):
        z = (np.arange(n, dtype=np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def gauge_sign_weights(n):
    """w_i = u_i - 1/2 with u_i = (top 53 bits of SplitMix64 output i) * 2^-53."""
    z = splitmix64(n)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 0.5


def contract_except(T, vecs, keep_axis):
    """Contract every axis of T except keep_axis with the given vectors."""
    out = T
    for ax in range(T.ndim - 1, -1, -1):
        if ax == keep_axis:
            continue
        out = np.tensordot(out, vecs[ax], axes=([ax], [0]))
    return out


def contract_all(T, vecs):
    out = T
    for ax in range(T.ndim - 1, -1, -1):
        out = np.tensordot(out, vecs[ax], axes=([ax], [0]))
    return float(out)


# --------------------------------------------------------------------------

class OperatorNetwork:
    """Pauli-basis operator network of Z_c(t) on an open Lx x Ly lattice."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self.lat = Lattice(cfg.Lx, cfg.Ly)
        self.centre = self.lat.centre() if cfg.centre is None else cfg.centre
        # The ZZ-coupling, X-field model is the paper's model conjugated by a
        # Hadamard on every site: H_zzx = W H W with W = prod_v Hd_v, and its
        # observable Z_c maps to W Z_c W = X_c.  So its C(t) is the paper-frame
        # network started from X_c and pinned on X at the observable site; the
        # gates (and their Trotter splitting) are the paper's.
        if cfg.model_axes not in ("paper", "zzx"):
            raise ValueError("model_axes is 'paper' or 'zzx'")
        self.obs_p = 3 if cfg.model_axes == "paper" else 1
        self.G1 = field_ptm(cfg.h, cfg.dt)
        self.G2 = coupling_ptm(cfg.J, cfg.dt)
        self.reset()

    # -- state ---------------------------------------------------------------
    def reset(self):
        """t = 0: psi_c = e_Z, psi_v = e_I elsewhere, all bonds chi = 1, mu = [[1]]."""
        lat = self.lat
        self.chi = [1] * lat.n_bonds
        self.psi = []
        for v in range(lat.n_sites):
            T = np.zeros((1,) * lat.degree(v) + (4,))
            T[(0,) * lat.degree(v) + (self.obs_p if v == self.centre else 0,)] = 1.0
            self.psi.append(T)
        self.M = [[np.ones((1, 1)), np.ones((1, 1))] for _ in range(lat.n_bonds)]
        self.lam = [np.ones(1) for _ in range(lat.n_bonds)]
        self.step_count = 0
        self.layer_gate_err = 0.0
        self.layer_flags = 0
        self.last_gauge = (0, 0.0)

    def site_dims(self, v):
        return tuple(self.chi[b] for (_, _, b) in self.lat.legs[v]) + (4,)

    def incoming(self, b, v):
        """Gauge message on bond b travelling into site v."""
        v1, v2, _ = self.lat.bonds[b]
        src = v2 if v == v1 else v1
        return self.M[b][self.lat.direction(b, src)]

    # -- a1: field half-step -----------------------------------------------------
    def apply_field(self):
        """psi_v[.., p'] = sum_p G1[p', p] psi_v[.., p] on every site."""
        for v in range(self.lat.n_sites):
            self.psi[v] = np.tensordot(self.psi[v], self.G1, axes=([-1], [1]))

    # -- a2..a7: two-site gate ----------------------------------------------------
    def gate_update(self, b):
        cfg, lat = self.cfg, self.lat
        v1, v2, _ = lat.bonds[b]
        chi_cut = self.chi[b]
        flags = 0
        sides = []
        for v in (v1, v2):
            legs = lat.legs[v]
            cut_pos = lat.leg_position(v, b)
            T = self.psi[v]
            env = []
            for pos, (_, u, be) in enumerate(legs):
                if be == b:
                    continue
                S, Sinv, ncut = pseudo_sqrt(self.incoming(be, v), cfg.eps_pinv)
                if ncut:
                    flags |= FLAG_PINV_CUT
                T = mode_product(T, S, pos)               # absorb (cv_i)
                env.append((pos, Sinv))
            order = [pos for pos, _ in env] + [cut_pos, len(legs)]
            X = np.transpose(T, order)                      # [env.., cut, p]
            env_dims = X.shape[:-2]
            m = int(np.prod(env_dims)) if env_dims else 1
            n = chi_cut * 4
            Xm = X.reshape((m, n), order="F")               # rows env, cols c + chi*p
            Q, R = np.linalg.qr(Xm)
            sgn = np.sign(np.diag(R))
            sgn[sgn == 0] = 1.0
            R = sgn[:, None] * R
            Q = Q * sgn[None, :]
            k = R.shape[0]
            R3 = R.reshape((k, chi_cut, 4), order="F")     # R3[k, c, d] = R[k, c + chi*d]
            sides.append(dict(v=v, order=order, env=env, env_dims=env_dims, m=m, Q=Q, R3=R3, k=k))
        A, B = sides
        # bond matrix over the cut, then the gate on the Pauli pair
        Theta = np.einsum("acd,bce->adbe", A["R3"], B["R3"])        # [k1, d1, k2, d2]
        G4 = self.G2.reshape(4, 4, 4, 4)                            # [e1, e2, d1, d2]
        Thp = np.einsum("xyde,adbe->axby", G4, Theta)               # [k1, e1, k2, e2]
        k1, k2 = A["k"], B["k"]
        U, s, Vt = np.linalg.svd(Thp.reshape(k1 * 4, k2 * 4), full_matrices=False)
        if not (s[0] > 0.0) or not np.all(np.isfinite(s)):
            raise FloatingPointError("bond matrix is zero or not finite")
        nkeep = int(np.count_nonzero(s >= cfg.eps_cut * s[0]))
        chi_new = min(nkeep, cfg.chi_max)
        if chi_new < len(s) and s[chi_new - 1] - s[chi_new] <= 1e-10 * s[0] and chi_new == cfg.chi_max:
            flags |= FLAG_DEGENERATE_CUT
        sk = s[:chi_new]
        lam = sk / math.sqrt(math.fsum(sk * sk))
        gate_err = math.fsum(s[chi_new:] ** 2) / math.fsum(s ** 2)
        rs = np.sqrt(sk)
        M1 = U[:, :chi_new].reshape(k1, 4, chi_new) * rs[None, None, :]      # [k1, e1, j]
        M2 = Vt[:chi_new, :].T.reshape(k2, 4, chi_new) * rs[None, None, :]   # [k2, e2, j]
        cv1 = np.einsum("mk,kej->mje", A["Q"], M1, optimize=True)                         # [m1, j, p]
        w = gauge_sign_weights(A["m"] * 4).reshape((A["m"], 4), order="F")
        t = np.einsum("mje,me->j", cv1, w, optimize=True)
        flip = t < 0
        cv1[:, flip, :] *= -1.0
        M2[:, :, flip] *= -1.0
        cv2 = np.einsum("mk,kej->mje", B["Q"], M2, optimize=True)
        for side, cv in ((A, cv1), (B, cv2)):
            T = cv.reshape(tuple(side["env_dims"]) + (chi_new, 4), order="F")
            T = np.transpose(T, np.argsort(side["order"]))              # inverse permute
            for pos, Sinv in side["env"]:
                T = mode_product(T, Sinv, pos)                           # deabsorb
            self.psi[side["v"]] = np.ascontiguousarray(T)
        self.chi[b] = chi_new
        D = np.diag(lam)
        self.M[b] = [D.copy(), D.copy()]
        self.lam[b] = lam
        return dict(chi_new=chi_new, s=s, lam=lam, gate_err=gate_err, flags=flags, flip=flip)

    # -- a8: gauge BP on the norm network -------------------------------------------
    def _norm_message(self, v, pos, M):
        """Unnormalised M_hat_{v -> w} for the leg at axis pos (Eq. bp, matrix form)."""
        psi = self.psi[v]
        T = psi
        for pos2, (_, u, bu) in enumerate(self.lat.legs[v]):
            if pos2 == pos:
                continue
            v1, v2, _ = self.lat.bonds[bu]
            T = mode_product(T, M[bu][self.lat.direction(bu, u)], pos2)
        axes = [a for a in range(psi.ndim) if a != pos]
        return np.tensordot(psi, T, axes=(axes, axes))

    def gauge_bp(self):
        cfg, lat = self.cfg, self.lat
        alpha = cfg.bp_alpha
        if cfg.bp_init == "uniform":
            self.M = [[np.eye(c) / math.sqrt(c), np.eye(c) / math.sqrt(c)] for c in self.chi]
        sweeps, delta = 0, float("inf")
        bethe_logs = None
        while sweeps < cfg.bp_max_sweeps:
            new = {}
            for v in range(lat.n_sites):
                for pos, (_, w, be) in enumerate(lat.legs[v]):
                    new[(be, lat.direction(be, v))] = self._norm_message(v, pos, self.M)
            # Bethe estimate of sum_p psi.psi for the message set of this sweep
            logs, sgn = [], 1.0
            for v in range(lat.n_sites):
                _, w, be = lat.legs[v][0]
                f = float(np.sum(new[(be, lat.direction(be, v))] * self.M[be][lat.direction(be, w)]))
                logs.append(math.log(abs(f)) if f != 0 else -math.inf)
                sgn *= math.copysign(1.0, f)
            for b in range(lat.n_bonds):
                z = float(np.sum(self.M[b][0] * self.M[b][1]))
                logs.append(-math.log(abs(z)) if z != 0 else math.inf)
                sgn *= math.copysign(1.0, z)
            bethe_logs = (logs, sgn)
            delta = 0.0
            upd = {}
            for (b, d), Mh in new.items():
                Mh = 0.5 * (Mh + Mh.T)
                nrm = math.sqrt(math.fsum((Mh * Mh).ravel()))
                if nrm > 0:
                    Mh = Mh / nrm
                Mo = self.M[b][d]
                Mn = (1.0 - alpha) * Mo + alpha * Mh
                nn = math.sqrt(math.fsum((Mn * Mn).ravel()))
                if nn > 0:
                    Mn = Mn / nn
                delta = max(delta, float(np.max(np.abs(Mn - Mo))))
                upd[(b, d)] = Mn
            for (b, d), Mn in upd.items():
                self.M[b][d] = Mn
            sweeps += 1
            if delta < cfg.bp_tol:
                break
        logs, sgn = bethe_logs if bethe_logs else ([0.0], 1.0)
        self.bethe_norm = sgn * math.exp(math.fsum(logs)) if all(np.isfinite(logs)) else float("nan")
        self.last_gauge = (sweeps, delta)
        return sweeps, delta

    # -- diagnostic: per-site non-identity Pauli weight ---------------------------------
    def pauli_weights(self):
        """BP estimate of n(r, t), the per-site non-identity Pauli weight of
        Sec. "Operator Spreading and Lightcone Saturation": with the gauge
        messages of the last gauge BP as the environment of every virtual leg,
        W_v[p, p'] = sum psi_v[.., p] (x_e M_{e -> v}) psi_v[.., p'] is the
        weight of the Pauli strings by their letter at v (exact on a tree with
        converged messages), and n_v = 1 - W_v[I, I] / tr W_v."""
        out = []
        for v in range(self.lat.n_sites):
            psi = self.psi[v]
            T = psi
            for pos, (_, u, bu) in enumerate(self.lat.legs[v]):
                T = mode_product(T, self.M[bu][self.lat.direction(bu, u)], pos)
            axes = list(range(psi.ndim - 1))
            W = np.tensordot(psi, T, axes=(axes, axes))
            out.append(1.0 - W[0, 0] / np.trace(W))
        return np.array(out)

    # -- a9: measurement BP and log-space Bethe -------------------------------------
    def pinned(self):
        out = []
        for v in range(self.lat.n_sites):
            p = self.obs_p if v == self.centre else 0
            out.append(self.psi[v][..., p])
        return out

    def measure(self, alpha=None):
        cfg, lat = self.cfg, self.lat
        if alpha is None:
            alpha = cfg.bp_alpha if cfg.meas_alpha is None else cfg.meas_alpha
        tol = cfg.bp_tol if cfg.meas_tol is None else cfg.meas_tol
        maxs = cfg.bp_max_sweeps if cfg.meas_max_sweeps is None else cfg.meas_max_sweeps
        T = self.pinned()
        m = [[np.ones(c) / math.sqrt(c), np.ones(c) / math.sqrt(c)] for c in self.chi]

        def incoming_vecs(v, msgs):
            out = []
            for (_, u, bu) in lat.legs[v]:
                out.append(msgs[bu][lat.direction(bu, u)])
            return out

        sweeps, delta = 0, float("inf")
        while sweeps < maxs:
            new = {}
            for v in range(lat.n_sites):
                vecs = incoming_vecs(v, m)
                for pos, (_, w, be) in enumerate(lat.legs[v]):
                    new[(be, lat.direction(be, v))] = contract_except(T[v], vecs, pos)
            delta = 0.0
            upd = {}
            for (b, d), mh in new.items():
                mo = m[b][d]
                nrm = math.sqrt(math.fsum(mh * mh))
                if nrm > 0:
                    mh = mh / nrm
                if math.fsum(mh * mo) < 0:
                    mh = -mh
                mn = (1.0 - alpha) * mo + alpha * mh
                nn = math.sqrt(math.fsum(mn * mn))
                if nn > 0:
                    mn = mn / nn
                delta = max(delta, float(np.max(np.abs(mn - mo))))
                upd[(b, d)] = mn
            for (b, d), mn in upd.items():
                m[b][d] = mn
            sweeps += 1
            if delta < tol:
                break
        flags = 0
        if delta >= tol:
            flags |= FLAG_BP_NOT_CONVERGED_MEAS
        if sweeps >= cfg.trap_sweeps and delta < tol:
            flags |= FLAG_TRAP_CANDIDATE
        vs = [contract_all(T[v], incoming_vecs(v, m)) for v in range(lat.n_sites)]
        Ze = [float(np.dot(m[b][0], m[b][1])) for b in range(lat.n_bonds)]
        C, log_abs, sign, f2 = bethe_log_sign(vs, Ze)
        flags |= f2
        self.meas_messages = m
        return dict(C=C, log_abs_C=log_abs, sign=sign, meas_sweeps=sweeps, meas_delta=delta,
                    flags=flags, vs=vs, Ze=Ze)


def spreading_stats(n, lat, centre):
    """The spreading measures of Sec. "Spatial operator spreading" from the
    per-site weights n(r): p(r) = n(r) / sum n, the mean Manhattan radius
    R_L1 = sum p |r - r_c|_1, the RMS Euclidean radius
    R_L2 = sqrt(sum p |r - r_c|_2^2) and the spatial entropy fraction
    S_frac = -sum p ln p / ln(number of sites) (Eq. sfrac; 0 ln 0 = 0)."""
    n = np.asarray(n, dtype=float)
    p = n / n.sum()
    cx, cy = lat.coords(centre)
    r1 = r2 = ent = 0.0
    for v in range(lat.n_sites):
        x, y = lat.coords(v)
        r1 += p[v] * (abs(x - cx) + abs(y - cy))
        r2 += p[v] * ((x - cx) ** 2 + (y - cy) ** 2)
        if p[v] > 0:
            ent -= p[v] * math.log(p[v])
    return r1, math.sqrt(r2), ent / math.log(lat.n_sites)


def bethe_log_sign(vs, Ze):
    """Eq. bethe: C = exp(sum log|vs| - sum log|Z_e|) * prod sign(vs) * prod sign(Z_e)."""
    flags = 0
    if any(v == 0.0 for v in vs):
        return 0.0, -math.inf, 0, FLAG_BETHE_ZERO
    if any(z == 0.0 for z in Ze):
        return float("nan"), float("nan"), 0, FLAG_BETHE_ZERO
    log_abs = math.fsum([math.log(abs(v)) for v in vs]) - math.fsum([math.log(abs(z)) for z in Ze])
    sign = 1
    for x in list(vs) + list(Ze):
        if x < 0:
            sign = -sign
    return sign * math.exp(log_abs), log_abs, sign, flags
