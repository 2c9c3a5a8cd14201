"""Tier-B: the FDP=H-approximated kernel, assembled densely (test infrastructure only).

This module builds the operator that the FDP=H method applies, one kernel
row K~_{i,:,:} at a time, directly from the paper's definitions, and applies
it by the same direct convolution as Tier-A.  It never uses rings, the shift
operator, sparse F/G matrices or any low-rank compression: it is the exact
dense form of what the method approximates.  A GPU FDP=H result differs from
it only by the low-rank (ACA) error and rounding.

Steps, in the paper's order:
  * clustering by recursive bisection of bounding boxes of element centres
    along the longest side (Sec. 2.3 and Sec. 4.2.2);
  * block cluster tree with the admissibility test diam < eta*dist (Eq. 8),
    where diam = box diagonal + longest element, i*, j* = box centres and
    dist = |i* - j*| - diam (Sec. 4.2.2); a block whose receiver or source
    cluster holds at most `leaf_size` elements is an inadmissible leaf (the
    stop rule of Eq. 9 expressed as a cluster size);
  * ART integers (Eq. 42 for the receiver shift; App. C.2 for the
    receiver-averaged travel-time step and the Domain-F duration, plus n_c
    steps of 2D broadening, Sec. 4.3 and App. H);
  * Domain F: amplitude K^F_ij over the pair's window (Eq. 51) times the
    degenerate waveform of the representative receiver (Eq. 50);
  * Domain S (admissible): static rate K^S_ij dt from the end of Domain F
    (App. B.1, with the decimal term removed by the App. C.2 choice);
  * Domain S transient (2D): temporal rank-2 reading K^S + K^tr h^tr with the
    temporal pivot at the start of Domain S (App. H.1, App. B.3), the
    waveform h^tr taken from the representative receiver and the source
    element nearest the source-box centre, and its length cut by the
    eps_Q / eps_st rule (App. A.1, App. H.1);
  * inadmissible leaves: exact kernel up to the window W_ij, then the static
    rate (App. E), W_ij chosen by the same eps_Q / eps_st rule.

On curved faults the method is applied per stress component and projected
on the receiver normal (Sec. 4.2.2 and App. F.2: "stress-then-project"); on
a planar fault the single component is the traction itself.

Parity: the integer steps are checked against brute-force and closed-form
properties (causality of every admissible pair, exactness of the travel-time
split on a line, the sum of each degenerate waveform equal to one, the tree
statistics of a planar fault); the all-near-field limit reproduces Tier-A to
rounding; the approximated kernel is checked against Tier-A within the
method's own error envelope (tests/test_oracle_fdph.py).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .kernel2d import Problem

SNAP = 1e-9


def _snap(v):
    """Snap values within 1e-9 (relative) of an integer onto it."""
    v = np.asarray(v, dtype=np.float64)
    r = np.round(v)
    return np.where(np.abs(v - r) <= SNAP * np.maximum(1.0, np.abs(v)), r, v)


def ifloor(v):
    """Floor of the travel-time steps of Eq. 42 and App. C.2 (a value within
    rounding of an integer counts as that integer)."""
    return np.floor(_snap(v)).astype(np.int64)


def iceil(v):
    """Ceiling of the Domain-F end step of App. C.2 (snapped as ifloor)."""
    return np.ceil(_snap(v)).astype(np.int64)


@dataclass
class FdphParams:
    """eta of the admissibility test (Eq. 8); the leaf size that stands in for
    the stop rule of Eq. 9; eps_q / eps_st of the static cut-off rule (App. A.1,
    App. H.1); n_c steps of Domain-F broadening (Sec. 4.3, App. H); the
    optional staircase transient (App. A.1 applied to h^tr, App. B.3)."""

    eta: float = 2.0
    leaf_size: int = 32
    eps_q: float = 1e-3
    eps_st: float = 1e-6
    n_c: int = 20
    quantize_tr: bool = False  # staircase transient waveform (App. A.1 applied to h^tr, App. B.3)
    eps_q_tr: float = 0.1      # relative bound of that staircase


def quantize_staircase(h, eps_rel, eps_abs):
    """Partition of the lags of h into runs represented by one value each.

    Quantization (App. A.1): starting at b_0 = 0, each run [b_q, b_{q+1}) is the
    longest one whose representative, the mean of its first and last values
    (the paper's choice for the anti-plane runs), stays within
    min(eps_rel |h^_q|, eps_abs) of every value in the run.  Returns the run
    starts b (with b_Q = len(h) appended) and the representatives h^.
    """
    h = np.asarray(h, dtype=np.float64)
    n = len(h)
    b = [0]
    rep = []
    start = 0
    while start < n:
        end = start + 1
        lo = hi = h[start]
        best_rep = h[start]
        while end < n:
            lo2 = min(lo, h[end])
            hi2 = max(hi, h[end])
            r = 0.5 * (h[start] + h[end])
            tol = min(eps_rel * abs(r), eps_abs)
            if max(hi2 - r, r - lo2) > tol:
                break
            lo, hi, best_rep = lo2, hi2, r
            end += 1
        rep.append(best_rep)
        b.append(end)
        start = end
    return np.array(b, dtype=np.int64), np.array(rep)


@dataclass
class Cluster:
    """Node of the cluster tree (Sec. 2.3): the bounding box of its element
    centres and the elements it holds."""

    lo: np.ndarray
    hi: np.ndarray
    idx: np.ndarray
    level: int
    children: list = field(default_factory=list)

    @property
    def center(self):
        """Box centre: the representative point i* or j* (Sec. 4.2.2)."""
        return 0.5 * (self.lo + self.hi)

    @property
    def diag(self):
        """Box diagonal, the geometric part of diam (Sec. 4.2.2)."""
        return float(np.hypot(*(self.hi - self.lo)))

    @property
    def is_leaf(self):
        """Not split further (Sec. 2.3)."""
        return not self.children


def build_cluster_tree(centers, leaf_size):
    """Cluster tree (Sec. 2.3): recursive bisection of the bounding box along
    its longest side.

    Ties between sides go to the lower axis; centres at or below the split
    coordinate go to the first child; empty children are dropped.
    """
    centers = np.asarray(centers, dtype=np.float64)
    idx = np.arange(centers.shape[0])
    root = Cluster(centers.min(axis=0), centers.max(axis=0), idx, 0)
    stack = [root]
    while stack:
        c = stack.pop()
        if len(c.idx) <= leaf_size or c.level >= 60:
            continue
        ext = c.hi - c.lo
        ax = 0 if ext[0] >= ext[1] else 1
        mid = 0.5 * (c.lo[ax] + c.hi[ax])
        sel = centers[c.idx, ax] <= mid
        lo_hi = c.hi.copy()
        lo_hi[ax] = mid
        hi_lo = c.lo.copy()
        hi_lo[ax] = mid
        kids = []
        if sel.any():
            kids.append(Cluster(c.lo.copy(), lo_hi, c.idx[sel], c.level + 1))
        if (~sel).any():
            kids.append(Cluster(hi_lo, c.hi.copy(), c.idx[~sel], c.level + 1))
        c.children = kids
        stack.extend(reversed(kids))
    return root


@dataclass
class Leaf:
    """Leaf of the block cluster tree (Sec. 2.3): receiver cluster tau, source
    cluster sigma, admissibility (Eq. 8) and, for an admissible leaf, its ART
    integers (Eq. 42, App. C.2) and waveforms (Eq. 50, App. H.1), filled on
    first use."""

    tau: Cluster
    sigma: Cluster
    admissible: bool
    diam: float
    dist: float
    # admissible-leaf data (filled lazily)
    mbar: np.ndarray = None   # [Ns] receiver-averaged travel-time step
    dm: np.ndarray = None     # [Ns] Domain-F duration in steps (incl. n_c)
    h: list = None            # per component: [Ns][max dm] degenerate waveform
    jpiv: int = -1            # source element of the transient pivot
    htr: list = None          # per component: transient waveform
    ntr: list = None          # per component: transient length
    nq_tr: list = None        # per component: staircase runs (0 when not quantized)


def build_block_tree(root, prob: Problem, eta, leaf_size):
    """Block cluster tree (Sec. 2.3): a cluster pair is an admissible leaf when
    diam < eta * dist (Eq. 8, with diam and dist of Sec. 4.2.2), an
    inadmissible leaf when either cluster is not split further, and is split
    into the pairs of its children otherwise."""
    leaves = []
    stack = [(root, root)]
    length = prob.length
    while stack:
        tau, sig = stack.pop()
        diag = max(tau.diag, sig.diag)
        maxlen = max(length[tau.idx].max(), length[sig.idx].max())
        diam = diag + maxlen
        rbar = float(np.hypot(*(tau.center - sig.center)))
        dist = rbar - diam
        if diam < eta * dist:
            leaves.append(Leaf(tau, sig, True, diam, dist))
        elif tau.is_leaf or sig.is_leaf:
            leaves.append(Leaf(tau, sig, False, diam, dist))
        else:
            for a in reversed(tau.children):
                for b in reversed(sig.children):
                    stack.append((a, b))
    return leaves


class FdphOracle:
    """Dense assembly of the FDP=H-approximated kernel (Tier-B), leaf by leaf:
    Secs. 3-5 and Apps. B.1, B.3, C.2, E, H."""

    def __init__(self, prob: Problem, M: int, params: FdphParams = FdphParams()):
        if prob.eps_t != 1.0:
            raise ValueError("the FDP=H time discretization assumes eps_t = 1 (Sec. 4.3)")
        self.prob = prob
        self.M = M
        self.p = params
        self.c = prob.beta  # anti-plane: only S waves
        self.cdt = self.c * prob.dt
        nrm = prob.normal
        if np.allclose(nrm, nrm[0], atol=1e-12, rtol=0):
            self.comp = [nrm[0].copy()]          # planar: traction itself
        else:
            self.comp = [np.array([1.0, 0.0]), np.array([0.0, 1.0])]
        self.root = build_cluster_tree(prob.center, params.leaf_size)
        self.leaves = build_block_tree(self.root, prob, params.eta, params.leaf_size)
        self.tol_abs = params.eps_st * prob.self_term()
        self._recv_leaves = None

    # -- statistics --------------------------------------------------------
    def stats(self):
        """Leaf and pair counts of the block cluster tree (Sec. 2.3)."""
        adm = [l for l in self.leaves if l.admissible]
        inad = [l for l in self.leaves if not l.admissible]
        return dict(
            n_adm=len(adm),
            n_inadm=len(inad),
            sum_nr_ns_adm=int(sum(len(l.tau.idx) + len(l.sigma.idx) for l in adm)),
            near_pairs=int(sum(len(l.tau.idx) * len(l.sigma.idx) for l in inad)),
        )

    # -- component kernels ---------------------------------------------------
    def comp_step(self, c, P, j, t):
        """Step response of stress component c at points P from sources j (on a
        curved fault the components are approximated separately, App. F.2)."""
        sx, sy = self.prob.stress_step(P, j, t)
        e = self.comp[c]
        return sx * e[0] + sy * e[1]

    def comp_static(self, c, P, j):
        """Static stress rate of component c: the late-time limit that Domain S
        keeps (App. B.1)."""
        sx, sy = self.prob.stress_static(P, j)
        e = self.comp[c]
        return sx * e[0] + sy * e[1]

    def comp_kernel(self, c, P, j, m):
        """K_m of component c: the step response differenced over one step (the
        definition under Eq. 4, eps_t = 1)."""
        dt = self.prob.dt
        m = np.asarray(m, dtype=np.float64)
        return self.comp_step(c, P, j, (m + 1.0) * dt) - self.comp_step(c, P, j, m * dt)

    def recv_weight(self, c, i):
        """Weight of component c in receiver i's traction: its normal (App. F.2)."""
        e = self.comp[c]
        return self.prob.normal[i, 0] * e[0] + self.prob.normal[i, 1] * e[1]

    # -- ART integers ----------------------------------------------------------
    def art_delta_m(self, leaf, i):
        """delta m_i = floor((r_{i j*} - r_{i* j*}) / (c dt)), Eq. 42."""
        d = self.prob.center[i] - leaf.sigma.center
        r_ij = np.hypot(d[..., 0], d[..., 1])
        rbar = float(np.hypot(*(leaf.tau.center - leaf.sigma.center)))
        return ifloor((r_ij - rbar) / self.cdt)

    def art_source(self, leaf):
        """(mbar_j, dm_j) of App. C.2 plus n_c broadening, for j in sigma."""
        if leaf.mbar is None:
            js = leaf.sigma.idx
            r = np.hypot(*(self.prob.center[js] - leaf.tau.center).T)
            half = self.prob.half[js]
            mbar = ifloor((r - half) / self.cdt)
            mend = iceil((r + half) / self.cdt)
            leaf.mbar = mbar
            leaf.dm = mend - mbar + self.p.n_c
        return leaf.mbar, leaf.dm

    def waveforms(self, leaf):
        """Degenerate waveforms h_{a,j,m} (Eq. 50) for every component."""
        if leaf.h is None:
            mbar, dm = self.art_source(leaf)
            js = leaf.sigma.idx
            istar = leaf.tau.center
            L = int(dm.max())
            mm = mbar[:, None] + np.arange(L)[None, :]
            valid = np.arange(L)[None, :] < dm[:, None]
            hs = []
            for c in range(len(self.comp)):
                Kw = self.comp_kernel(c, istar, js[:, None], mm)
                Kw = np.where(valid, Kw, 0.0)
                amp = Kw.sum(axis=1)
                with np.errstate(divide="ignore", invalid="ignore"):
                    h = np.where(np.abs(amp)[:, None] > 0, Kw / amp[:, None], 0.0)
                hs.append(h)
            leaf.h = hs
        return leaf.h

    def cutoff(self, series, ref_static):
        """Length after which |series| stays within min(eps_Q|ref|, eps_st K_0).

        Implements the eps_Q / eps_st rule of App. A.1 and App. H.1: returns
        1 + the last index violating the bound (0 if none does).
        """
        tol = min(self.p.eps_q * abs(ref_static), self.tol_abs)
        bad = np.nonzero(np.abs(series) > tol)[0]
        return 0 if bad.size == 0 else int(bad[-1]) + 1

    def transient(self, leaf):
        """Leaf-level transient waveform h^tr and its length, per component
        (temporal rank 2 of App. H.1 with the pivot at the start of Domain S,
        App. B.3; length by the rule of App. A.1)."""
        if leaf.htr is None:
            mbar, dm = self.art_source(leaf)
            js = leaf.sigma.idx
            jst = leaf.sigma.center
            d = np.hypot(*(self.prob.center[js] - jst).T)
            k = int(np.argmin(d))  # first minimum: lowest index on ties
            jp = int(js[k])
            leaf.jpiv = jp
            s0 = int(mbar[k] + dm[k])
            istar = leaf.tau.center
            dt = self.prob.dt
            htr, ntr, nq = [], [], []
            for c in range(len(self.comp)):
                if s0 >= self.M:
                    htr.append(np.zeros(0))
                    ntr.append(0)
                    nq.append(0)
                    continue
                ks = np.arange(self.M - s0)
                ks_static = self.comp_static(c, istar, jp) * dt
                series = self.comp_kernel(c, istar, jp, s0 + ks) - ks_static
                n = self.cutoff(series, ks_static)
                if n == 0 or series[0] == 0.0:
                    htr.append(np.zeros(0))
                    ntr.append(0)
                    nq.append(0)
                    continue
                hh = series[:n] / series[0]
                runs = 0
                if self.p.quantize_tr:
                    # absolute bound of the kernel values in units of the
                    # pivot amplitude: |K^tr (h - h^)| <= eps_st mu/(2 beta)
                    b, rep = quantize_staircase(hh, self.p.eps_q_tr, self.tol_abs / abs(series[0]))
                    hh = np.repeat(rep, np.diff(b))
                    runs = len(rep)
                htr.append(hh)
                ntr.append(n)
                nq.append(runs)
            leaf.htr, leaf.ntr, leaf.nq_tr = htr, ntr, nq
        return leaf.htr, leaf.ntr

    def transient_amplitude(self, c, P, js, tplus, kst):
        """K^tr_ij: the pair's deviation from the static rate over the first
        step of its Domain S, taken in the pair's own continuous time frame,
        the step (t+_ij, t+_ij + dt) that follows its Domain-F window (the
        window of Eq. 28): S_ij(t+ + dt) - S_ij(t+) - K^S_ij dt.  At the
        representative receiver this is the temporal pivot of the transient
        waveform (App. H.1, temporal rank 2)."""
        dt = self.prob.dt
        return self.comp_step(c, P, js, tplus + dt) - self.comp_step(c, P, js, tplus) - kst

    def near_window(self, i, js):
        """W_ij for the near pairs (App. E with the eps_Q / eps_st rule)."""
        M = self.M
        dt = self.prob.dt
        W = np.empty(len(js), dtype=np.int64)
        Kfull = self.prob.kernel(i, js[:, None], np.arange(M)[None, :])
        ks = self.prob.traction_static(i, js) * dt
        for k in range(len(js)):
            W[k] = self.cutoff(Kfull[k] - ks[k], ks[k])
        return W, Kfull, ks

    # -- receiver rows --------------------------------------------------------
    def receiver_leaves(self, i):
        """Leaves whose receiver cluster holds receiver i (Sec. 2.3)."""
        if self._recv_leaves is None:
            self._recv_leaves = {}
            for a, lf in enumerate(self.leaves):
                for r in lf.tau.idx:
                    self._recv_leaves.setdefault(int(r), []).append(a)
        return self._recv_leaves.get(int(i), [])

    def f_window(self, lf, i):
        """The pair's own Domain-F window (t-_ij, t+_ij) for receiver i and the
        sources of admissible leaf lf: the travel time r_ij / c less the lead
        r_{i*j} / c - mbar_j dt of the representative receiver's window, and
        plus its tail (mbar_j + dm_j) dt - r_{i*j} / c (Eqs. 28-29 with the
        discretized mbar_j dt and dm_j dt of App. C.2)."""
        mbar, dm = self.art_source(lf)
        js = lf.sigma.idx
        dt = self.prob.dt
        r_ij = np.hypot(*(self.prob.center[js] - self.prob.center[i]).T)
        r_sj = np.hypot(*(self.prob.center[js] - lf.tau.center).T)
        tminus = r_ij / self.c - (r_sj / self.c - mbar * dt)
        tplus = r_ij / self.c + ((mbar + dm) * dt - r_sj / self.c)
        return tminus, tplus

    def leaf_block(self, i, a, n_lags=None, pieces=("F", "S", "tr")):
        """K~_{i,j,k} for the sources j of leaf a (a holds receiver i): (js, [Ns][L]):
        inadmissible leaves by App. E, admissible ones as the sum of Domain F
        (Eqs. 50-51), Domain S (App. B.1) and the 2D transient (App. H.1).

        L = min(M, n_lags): only the first L lags are evaluated (the operator
        itself, windows and transient lengths included, is the M-lag one).
        `pieces` selects the terms of an admissible leaf that are summed
        (Domain F, Domain S static, transient); all by default.
        """
        prob, dt = self.prob, self.prob.dt
        M = self.M if n_lags is None else min(self.M, int(n_lags))
        P = prob.center[i]
        ks = np.arange(M)
        lf = self.leaves[a]
        js = lf.sigma.idx
        if not lf.admissible:
            W, Kfull, kst = self.near_window(i, js)
            Kfull = Kfull[:, :M]
            return js, np.where(ks[None, :] < W[:, None], Kfull, kst[:, None])
        out = np.zeros((len(js), M))
        mbar, dm = self.art_source(lf)
        dmi = int(self.art_delta_m(lf, i))
        hs = self.waveforms(lf)
        htr, ntr = self.transient(lf)
        tminus, tplus = self.f_window(lf, i)
        start = dmi + mbar            # first lag of Domain F (ART)
        sstart = start + dm           # first lag of Domain S
        for c in range(len(self.comp)):
            w = self.recv_weight(c, i)
            if w == 0.0:
                continue
            amp = self.comp_step(c, P, js, tplus) - self.comp_step(c, P, js, tminus)
            kst = self.comp_static(c, P, js) * dt
            blk = np.zeros((len(js), M))
            # Domain F
            if "F" in pieces:
                h = hs[c]
                kk = ks[None, :] - start[:, None]
                inF = (kk >= 0) & (kk < dm[:, None])
                hv = np.take_along_axis(h, np.clip(kk, 0, h.shape[1] - 1), axis=1)
                blk += np.where(inF, amp[:, None] * hv, 0.0)
            # Domain S static
            if "S" in pieces:
                blk += np.where(ks[None, :] >= sstart[:, None], kst[:, None], 0.0)
            # Domain S transient (2D)
            if ntr[c] > 0 and "tr" in pieces:
                ktr_amp = self.transient_amplitude(c, P, js, tplus, kst)
                kt = ks[None, :] - sstart[:, None]
                inT = (kt >= 0) & (kt < ntr[c])
                tv = htr[c][np.clip(kt, 0, ntr[c] - 1)]
                blk += np.where(inT, ktr_amp[:, None] * tv, 0.0)
            out += w * blk
        return js, out

    def row(self, i):
        """K~_{i,j,k} for all sources j and lags k < M (float64 [N][M]): the sum
        over the leaves of receiver i's row of the block cluster tree (Sec. 2.3)."""
        out = np.zeros((self.prob.n, self.M))
        for a in self.receiver_leaves(i):
            js, blk = self.leaf_block(i, a)
            out[js] += blk
        return out

    def rows(self, receivers):
        """row() of several receivers: [R][N][M]."""
        return np.stack([self.row(i) for i in receivers])

    def apply_at(self, i, D, steps):
        """T~_{i,n} for n in `steps` (the direct sum of Eq. 4 with K~)."""
        D = np.asarray(D, dtype=np.float64)
        out = np.zeros(len(steps))
        for a in self.receiver_leaves(i):
            js, blk = self.leaf_block(i, a, n_lags=max(steps) + 1)
            for k, n in enumerate(steps):
                L = min(n, self.M - 1) + 1
                out[k] += np.einsum("jm,mj->", blk[:, :L], D[n - np.arange(L)][:, js])
        return out

    # -- checks ----------------------------------------------------------------
    def causality_margin(self):
        """min over admissible leaves of min_i dm_i + min_j mbar_j (App. D.1)."""
        best = None
        for lf in self.leaves:
            if not lf.admissible:
                continue
            mbar, _ = self.art_source(lf)
            dmi = self.art_delta_m(lf, lf.tau.idx)
            v = int(np.min(dmi) + np.min(mbar))
            best = v if best is None else min(best, v)
        return best
