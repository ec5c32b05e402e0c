"""The sampled block matrix product, step by step, in float64 (oracle side).

Test infrastructure only (see the package docstring).

Notation follows the paper: M is m x n, N is n x p, the inner dimension is cut
into K contiguous blocks with sizes n_k (off[k] .. off[k+1]); M^k, N_k are the
k-th column block of M and row block of N; M^(i) is column i of M and N_(i)
row i of N; a_i = ||M^(i)||_2, b_i = ||N_(i)||_2, s_k = sum_{i in k} a_i b_i.

Two sampling modes share one description. An *atom* is a contiguous range of
the inner dimension; a *stratum* is a contiguous range of atoms that receives
its own number of draws c_s:

* ``block``      atoms are the K blocks, one stratum, c draws (the block
                 samplers the paper compares with: probabilities (1.2) or
                 (1.4), or uniform);
* ``stratified`` atoms are single inner indices, the K blocks are the
                 strata, block k gets c_k draws (the paper's Alg. 2 with
                 within-block probabilities (3.8) or uniform, and block sizes
                 uniform c/K, (4.2) or (3.9); or Alg. 3, whose block sizes
                 (4.7) come from a pilot sketch).

Alg. 1 (probabilities (1.1)) is either mode with K = 1 block of unit atoms.
"""

import math
from dataclasses import dataclass, field

import numpy as np

from .sampling import (quantize_weights, inclusive_cdf, draw_atoms,
                       allocate_draws)
from .rng import TAG_SAMPLE, TAG_PILOT

MODES = ("block", "stratified")
PROB_RULES = ("uniform", "norm", "exact", "user")
ALLOC_RULES = ("uniform", "norm", "opt", "user", "two_step")
PILOT_RULES = ("uniform", "norm")


# ----------------------------------------------------------------------------
# Partition
# ----------------------------------------------------------------------------

def check_partition(off, n):
    """Block offsets 0 = off[0] < off[1] < ... < off[K] = n (Alg. 2 input:
    sizes n_k >= 1 summing to n)."""
    off = [int(x) for x in off]
    if len(off) < 2 or off[0] != 0 or off[-1] != n:
        raise ValueError("partition must start at 0 and end at n")
    for a, b in zip(off[:-1], off[1:]):
        if b <= a:
            raise ValueError("block sizes must be positive")
    return off


# ----------------------------------------------------------------------------
# Norms (inputs of (1.1), (1.4), (3.8), (4.2))
# ----------------------------------------------------------------------------

def column_row_sq(M, N, chunk=8192):
    """col_sq[i] = ||M^(i)||_2^2 and row_sq[i] = ||N_(i)||_2^2 in float64.

    Each column (row) is promoted to float64 and its squares summed; large
    inputs are processed a slab of whole columns (rows) at a time, which does
    not change any single sum.
    """
    m, n = M.shape
    n2, p = N.shape
    if n2 != n:
        raise ValueError("inner dimensions differ")
    col_sq = np.empty(n, dtype=np.float64)
    row_sq = np.empty(n, dtype=np.float64)
    for j0 in range(0, n, chunk):
        blk = np.asarray(M[:, j0:j0 + chunk], dtype=np.float64)
        col_sq[j0:j0 + chunk] = np.einsum("hi,hi->i", blk, blk)
        blk = np.asarray(N[j0:j0 + chunk, :], dtype=np.float64)
        row_sq[j0:j0 + chunk] = np.einsum("if,if->i", blk, blk)
    return col_sq, row_sq


@dataclass
class BlockStats:
    """Per-block statistics: ||M^k||_F^2, ||N_k||_F^2 and s_k."""
    m_sq: np.ndarray
    n_sq: np.ndarray
    s: np.ndarray


def block_stats(col_sq, row_sq, off):
    """||M^k||_F^2 = sum of col_sq over block k, ||N_k||_F^2 likewise, and
    s_k = sum_{i in k} ||M^(i)||_2 ||N_(i)||_2 (the numerator of (4.2) and
    the denominator of (3.8)). Sums are correctly rounded (math.fsum)."""
    K = len(off) - 1
    ab = np.sqrt(col_sq * row_sq)
    m_sq = np.array([math.fsum(col_sq[off[k]:off[k + 1]]) for k in range(K)])
    n_sq = np.array([math.fsum(row_sq[off[k]:off[k + 1]]) for k in range(K)])
    s = np.array([math.fsum(ab[off[k]:off[k + 1]]) for k in range(K)])
    return BlockStats(m_sq, n_sq, s)


def block_product_sq(M, N, off, blocks=None):
    """||M^k N_k||_F^2 for each block k (or for the listed ``blocks``):
    the quantity (1.2) and (3.9) need, formed by multiplying the two blocks
    out in float64."""
    ks = range(len(off) - 1) if blocks is None else blocks
    out = []
    for k in ks:
        a = np.asarray(M[:, off[k]:off[k + 1]], dtype=np.float64)
        b = np.asarray(N[off[k]:off[k + 1], :], dtype=np.float64)
        x = a @ b
        out.append(float(np.sum(x * x)))
    return np.array(out)


# ----------------------------------------------------------------------------
# Design: probabilities and draw counts
# ----------------------------------------------------------------------------

@dataclass
class Design:
    """A sampling design: atoms, strata, integer weights and draw counts.

    atom_lo/atom_hi  inner-index range of each atom (A atoms)
    strat_off        atoms of stratum s are strat_off[s] .. strat_off[s+1]
    W                quantized weights (Python ints), one per atom
    cdf              per stratum, the inclusive running sums of its W
    T                per stratum, the CDF total
    cs               draws per stratum (sum = c)
    """
    mode: str
    atom_lo: np.ndarray
    atom_hi: np.ndarray
    strat_off: list
    W: list
    cdf: list
    T: list
    cs: list
    w: np.ndarray = field(default=None)   # float weights before quantizing
    g: np.ndarray = field(default=None)   # float allocation weights

    @property
    def c(self):
        return int(sum(self.cs))

    def p_hat(self):
        """Sampled probability of each atom within its stratum, W / T."""
        out = np.zeros(len(self.W))
        for s in range(len(self.T)):
            for a in range(self.strat_off[s], self.strat_off[s + 1]):
                if self.T[s] > 0:
                    out[a] = float(self.W[a]) / float(self.T[s])
        return out


def atom_weights(mode, prob, off, col_sq, row_sq, stats, blkprod_sq=None,
                 user_w=None):
    """Float weights w_a, proportional to the sampling probabilities.

    block mode (atoms = blocks):
      uniform  w_k = 1                        (uniform block sampling)
      norm     w_k = ||M^k||_F ||N_k||_F       (1.4)
      exact    w_k = ||M^k N_k||_F             (1.2)
    stratified mode (atoms = inner indices):
      uniform  w_i = 1                        (p_{k_i} = 1/n_k, method UU)
      norm     w_i = ||M^(i)||_2 ||N_(i)||_2   (3.8); with one block this is
                                              (1.1), Alg. 1's probabilities
    user       the caller's weights
    """
    K = len(off) - 1
    n = off[-1]
    if prob == "user":
        if user_w is None:
            raise ValueError("user weights missing")
        w = np.asarray(user_w, dtype=np.float64).copy()
        want = K if mode == "block" else n
        if w.shape != (want,):
            raise ValueError("user weights have the wrong length")
        return w
    if mode == "block":
        if prob == "uniform":
            return np.ones(K)
        if prob == "norm":
            return np.sqrt(stats.m_sq * stats.n_sq)
        if prob == "exact":
            if blkprod_sq is None:
                raise ValueError("rule 'exact' needs ||M^k N_k||_F^2")
            return np.sqrt(np.asarray(blkprod_sq, dtype=np.float64))
    else:
        if prob == "uniform":
            return np.ones(n)
        if prob == "norm":
            return np.sqrt(col_sq * row_sq)
    raise ValueError(f"rule {prob!r} not available in {mode} mode")


def alloc_weights(alloc, stats, blkprod_sq=None, pilot_sq=None):
    """Float allocation weights g_k of the strata (stratified mode).

      uniform   g_k = 1                              (c_k = c/K, method UU)
      norm      g_k = s_k                            (4.2), method ONC
      opt       g_k = sqrt(max(0, s_k^2 - ||M^k N_k||_F^2))   (3.9), method OPL
      two_step  g_k = |s_k^2 - ||C^{0k} D_{0k}||_F^2|^(1/2)    (4.7), Alg. 3
                (methods ONU / ONMCNR): the pilot estimate replaces
                ||M^k N_k||_F^2 and the absolute value replaces the clamp,
                since the estimate may exceed s_k^2
    """
    K = len(stats.s)
    if alloc == "uniform":
        return np.ones(K)
    if alloc == "norm":
        return stats.s.copy()
    if alloc == "opt":
        if blkprod_sq is None:
            raise ValueError("rule 'opt' needs ||M^k N_k||_F^2")
        d = stats.s * stats.s - np.asarray(blkprod_sq, dtype=np.float64)
        return np.sqrt(np.maximum(d, 0.0))
    if alloc == "two_step":
        if pilot_sq is None:
            raise ValueError("rule 'two_step' needs the pilot estimates")
        d = stats.s * stats.s - np.asarray(pilot_sq, dtype=np.float64)
        return np.sqrt(np.abs(d))
    raise ValueError(f"allocation rule {alloc!r} unknown")


def make_design(mode, off, c, w, g=None, user_ck=None):
    """Quantize the weights per stratum, build the CDFs and the draw counts.

    block: one stratum holding the K block atoms, c_1 = c.
    stratified: stratum k holds the n_k unit atoms of block k; its draw
    count comes from the allocation weights ``g`` (or ``user_ck``).
    Quantization is done separately in each stratum (its own maximum).
    """
    if mode not in MODES:
        raise ValueError("unknown mode")
    K = len(off) - 1
    if c < 1:
        raise ValueError("c must be positive")
    if mode == "block":
        lo = np.array(off[:-1], dtype=np.int64)
        hi = np.array(off[1:], dtype=np.int64)
        strat_off = [0, K]
    else:
        n = off[-1]
        lo = np.arange(n, dtype=np.int64)
        hi = lo + 1
        strat_off = list(off)
    S = len(strat_off) - 1
    W, cdf, T = [], [], []
    for s in range(S):
        Ws = quantize_weights(w[strat_off[s]:strat_off[s + 1]])
        W.extend(Ws)
        cs_cdf = inclusive_cdf(Ws)
        cdf.append(cs_cdf)
        T.append(cs_cdf[-1] if cs_cdf else 0)
    if mode == "block":
        cs = [c if T[0] > 0 else 0]
    elif user_ck is not None:
        cs = [int(x) for x in user_ck]
        if len(cs) != S or sum(cs) != c or min(cs) < 0:
            raise ValueError("user draw counts must be K non-negative ints "
                             "summing to c")
        for s in range(S):
            if (T[s] > 0) != (cs[s] > 0):
                raise ValueError("user draw counts must be positive exactly "
                                 "on the strata with positive weight")
    else:
        G = quantize_weights(g)
        cs = allocate_draws(c, G, T)
    return Design(mode, lo, hi, strat_off, W, cdf, T, cs,
                  w=np.asarray(w, dtype=np.float64),
                  g=None if g is None else np.asarray(g, dtype=np.float64))


# ----------------------------------------------------------------------------
# Sampling (Alg. 1 step 1, applied per stratum as in Alg. 2 step 1)
# ----------------------------------------------------------------------------

@dataclass
class Draws:
    """The drawn atoms in concatenation order (stratum-major, draw order).

    atom   global atom index of each draw
    strat  stratum of each draw
    scale  1 / sqrt(c_s p_hat) applied to the column of C and row of D
    lo, width   inner-index range of the drawn atom
    col_off     column of C where each draw starts; col_off[-1] = L
    """
    atom: np.ndarray
    strat: np.ndarray
    scale: np.ndarray
    lo: np.ndarray
    width: np.ndarray
    col_off: np.ndarray

    @property
    def L(self):
        return int(self.col_off[-1])


def draw_scale(c_s, W_a, T_s):
    """1 / sqrt(c_s p) with p = W_a / T_s, the factor of Alg. 1 step 1(b)
    (and of (3.2)), in float64: p, c_s p, the square root and the
    reciprocal are each rounded once."""
    q = float(W_a) / float(T_s)
    return 1.0 / math.sqrt(float(c_s) * q)


def sample(design, seed, trial=0, tag=TAG_SAMPLE, forced=None):
    """Draw c_s atoms from each stratum s, independently and with
    replacement, with probability p_hat = W / T.

    ``forced`` (tests only) replaces the random local atom choices: a list,
    per stratum, of local atom indices.
    """
    atom, strat, scale = [], [], []
    for s in range(len(design.T)):
        cnt = design.cs[s]
        if cnt == 0:
            continue
        a0 = design.strat_off[s]
        if forced is not None:
            local = list(forced[s])
        else:
            local = draw_atoms(design.cdf[s], design.T[s], cnt, seed, trial,
                               s, tag)
        for la in local:
            a = a0 + la
            if design.W[a] == 0:
                raise ValueError("forced draw of a zero-weight atom")
            atom.append(a)
            strat.append(s)
            scale.append(draw_scale(cnt, design.W[a], design.T[s]))
    atom = np.array(atom, dtype=np.int64)
    lo = design.atom_lo[atom] if len(atom) else np.zeros(0, np.int64)
    width = (design.atom_hi[atom] - lo) if len(atom) else np.zeros(0, np.int64)
    col_off = np.concatenate([[0], np.cumsum(width)]).astype(np.int64)
    return Draws(atom, np.array(strat, dtype=np.int64),
                 np.array(scale, dtype=np.float64), lo, width, col_off)


# ----------------------------------------------------------------------------
# Sketch and product (Alg. 1 step 1(b); Alg. 2 steps 3-4; (3.2)-(3.3))
# ----------------------------------------------------------------------------

def sketch(M, N, draws):
    """C (m x L) and D (L x p): each draw contributes its atom's columns of M
    and rows of N, multiplied by its scale, placed side by side in draw
    order (Alg. 2 step 3 concatenates the per-block sketches)."""
    m, p = M.shape[0], N.shape[1]
    C = np.zeros((m, draws.L))
    D = np.zeros((draws.L, p))
    for t in range(len(draws.atom)):
        lo, wd, c0 = int(draws.lo[t]), int(draws.width[t]), int(draws.col_off[t])
        C[:, c0:c0 + wd] = np.asarray(M[:, lo:lo + wd], np.float64) * draws.scale[t]
        D[c0:c0 + wd, :] = np.asarray(N[lo:lo + wd, :], np.float64) * draws.scale[t]
    return C, D


def sketch_product(C, D):
    """CD, the estimate of MN (Alg. 2 step 4, (3.3))."""
    return C @ D


def exact_product(M, N):
    """MN in float64."""
    return np.asarray(M, np.float64) @ np.asarray(N, np.float64)


def judge(MN, CD):
    """err = ||MN - CD||_F and rel = err / ||MN||_F (rel = 0 when both are 0,
    +inf when only ||MN||_F is 0)."""
    d = MN - CD
    err2 = float(np.sum(d * d))
    mn2 = float(np.sum(MN * MN))
    err = math.sqrt(err2)
    if mn2 == 0.0:
        rel = 0.0 if err2 == 0.0 else math.inf
    else:
        rel = err / math.sqrt(mn2)
    return err, rel, err2, mn2


def sketch_entries(M, N, draws, rows, cols):
    """Selected entries of CD straight from (3.3): for each (h, f),
    sum over draws t of scale_t^2 * sum_{i in atom_t} M[h, i] N[i, f],
    in float64 (for checks at sizes where CD itself is too large)."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    out = np.zeros(len(rows))
    for t in range(len(draws.atom)):
        lo, wd = int(draws.lo[t]), int(draws.width[t])
        a = np.asarray(M[rows, lo:lo + wd], np.float64)
        b = np.asarray(N[lo:lo + wd, :][:, cols], np.float64).T
        out += draws.scale[t] ** 2 * np.sum(a * b, axis=1)
    return out


def exact_entries(M, N, rows, cols, chunk=8192):
    """Selected entries of MN in float64: (MN)[h, f] = sum_i M[h, i] N[i, f]."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    out = np.zeros(len(rows))
    n = M.shape[1]
    for i0 in range(0, n, chunk):
        a = np.asarray(M[rows, i0:i0 + chunk], np.float64)
        b = np.asarray(N[i0:i0 + chunk, :][:, cols], np.float64).T
        out += np.sum(a * b, axis=1)
    return out


# ----------------------------------------------------------------------------
# Pilot of the two-step algorithm (Alg. 3, step 1)
# ----------------------------------------------------------------------------

@dataclass
class Pilot:
    """Step 1 of Alg. 3: the pilot design and draws, and per block the
    squared Frobenius norm of the pilot estimate C^{0k} D_{0k} of M^k N_k."""
    design: Design
    draws: Draws
    pilot_sq: np.ndarray


def pilot(M, N, off, c0, pilot_prob, seed, trial=0, col_row=None, forced=None):
    """Alg. 3 step 1: in every block k, Alg. 1 with [c0/K] draws and the
    pilot probabilities p_{0k_i} (uniform 1/n_k for ONU, (3.8) for ONMCNR),
    giving C^{0k} (m x [c0/K]) and D_{0k}; then ||C^{0k} D_{0k}||_F^2.

    Readings: [c0/K] is the integer part, so c0 >= K is required; a block
    whose pilot weights are all zero (rule (3.8) on a block with M^k N_k's
    outer products all zero) gets no pilot draws and estimate 0; the draws
    read the Philox streams of tag TAG_PILOT, so they are independent of
    step 2's. ``forced`` (tests only) fixes the local draws per block.
    """
    n = M.shape[1]
    off = check_partition(off, n)
    K = len(off) - 1
    if pilot_prob not in PILOT_RULES:
        raise ValueError("pilot probabilities are 'uniform' or 'norm'")
    r = int(c0) // K
    if r < 1:
        raise ValueError("c0 must be at least the number of blocks")
    col_sq, row_sq = col_row if col_row is not None else column_row_sq(M, N)
    stats = block_stats(col_sq, row_sq, off)
    w0 = atom_weights("stratified", pilot_prob, off, col_sq, row_sq, stats)
    live = [bool(np.any(w0[off[k]:off[k + 1]] > 0)) for k in range(K)]
    ck0 = [r if live[k] else 0 for k in range(K)]
    pilot_sq = np.zeros(K)
    if sum(ck0) == 0:
        return Pilot(None, None, pilot_sq)
    design0 = make_design("stratified", off, sum(ck0), w0, user_ck=ck0)
    draws0 = sample(design0, seed, trial, tag=TAG_PILOT, forced=forced)
    C0, D0 = sketch(M, N, draws0)
    for k in range(K):
        cols = np.flatnonzero(draws0.strat == k)
        if len(cols) == 0:
            continue
        # unit atoms: draw t is sketch column col_off[t]
        sel = draws0.col_off[cols]
        Z = C0[:, sel] @ D0[sel, :]
        pilot_sq[k] = float(np.sum(Z * Z))
    return Pilot(design0, draws0, pilot_sq)


# ----------------------------------------------------------------------------
# Closed forms (Lemma 1, Thm 2 proof, Remark 2.2, Remark 2.3)
# ----------------------------------------------------------------------------

def atom_products_sq(M, N, design):
    """||X_a||_F^2 for every atom, X_a = M[:, atom] N[atom, :]; for a unit
    atom this is a_i^2 b_i^2 (the Frobenius norm of an outer product is the
    product of the two vector norms)."""
    out = np.empty(len(design.atom_lo))
    for a, (lo, hi) in enumerate(zip(design.atom_lo, design.atom_hi)):
        x = np.asarray(M[:, lo:hi], np.float64)
        y = np.asarray(N[lo:hi, :], np.float64)
        if hi - lo == 1:
            out[a] = float(np.sum(x * x)) * float(np.sum(y * y))
        else:
            z = x @ y
            out[a] = float(np.sum(z * z))
    return out


def expected_sq_error(M, N, design):
    """E ||MN - CD||_F^2 of the design, exactly:

        sum_s (1 / c_s) ( sum_{a in s} ||X_a||_F^2 / p_a - ||sum_{a in s} X_a||_F^2 )

    Summing the per-entry variance (3.7) over all entries (Remark 2.2; the
    first line of the proof of Thm 2 for unit atoms), with the probabilities
    p_a = W_a / T_s that are actually sampled.
    """
    xa = atom_products_sq(M, N, design)
    ph = design.p_hat()
    total = 0.0
    for s in range(len(design.T)):
        a0, a1 = design.strat_off[s], design.strat_off[s + 1]
        lo, hi = int(design.atom_lo[a0]), int(design.atom_hi[a1 - 1])
        z = np.asarray(M[:, lo:hi], np.float64) @ np.asarray(N[lo:hi, :], np.float64)
        blk = float(np.sum(z * z))
        if design.cs[s] == 0:
            if blk != 0.0 or np.any(xa[a0:a1] != 0.0):
                raise ValueError("stratum without draws has a nonzero product")
            continue
        acc = 0.0
        for a in range(a0, a1):
            if xa[a] == 0.0:
                continue
            if ph[a] == 0.0:
                raise ValueError("atom with nonzero product has p = 0 (biased)")
            acc += xa[a] / ph[a]
        total += (acc - blk) / design.cs[s]
    return total


def sum_variance_real(col_sq, row_sq, off, blkprod_sq, p, ck):
    """The sum over entries of the asymptotic variances for real-valued
    within-block probabilities p (length n) and real block sizes ck (length
    K): sum_k sum_i a_i^2 b_i^2 / (c_k p_{k_i}) - sum_k ||M^k N_k||_F^2 / c_k
    (first line of the proof of Thm 2)."""
    tot = 0.0
    for k in range(len(off) - 1):
        sl = slice(off[k], off[k + 1])
        ab2 = col_sq[sl] * row_sq[sl]
        pk = p[sl]
        nz = ab2 > 0
        tot += (math.fsum(ab2[nz] / pk[nz]) - blkprod_sq[k]) / ck[k]
    return tot


def optimal_value(stats, blkprod_sq, c):
    """(3.10): the minimum of the summed variance,
    (1/c) [ sum_k (1 - v_k^2)^(1/2) s_k ]^2 with v_k s_k = ||M^k N_k||_F."""
    s = stats.s
    v2 = np.where(s > 0, np.asarray(blkprod_sq) / np.where(s > 0, s * s, 1.0), 0.0)
    return (math.fsum(np.sqrt(np.maximum(1.0 - v2, 0.0)) * s)) ** 2 / c


# ----------------------------------------------------------------------------
# Probability error bounds (Thm 3.3 (3.11)-(3.12), Thm 4.2 (4.3)-(4.4),
# Thm 4.4 (4.8)-(4.9))
# ----------------------------------------------------------------------------

def sampled_beta(design, col_sq, row_sq):
    """The largest beta <= 1 with p_hat >= beta p for the probabilities (3.8)
    p_{k_i} = a_i b_i / s_k, over the atoms with p > 0 (stratified design)."""
    w = np.sqrt(np.asarray(col_sq, np.float64) * np.asarray(row_sq, np.float64))
    ph = design.p_hat()
    beta = 1.0
    for s in range(len(design.T)):
        a0, a1 = design.strat_off[s], design.strat_off[s + 1]
        ws = w[a0:a1]
        tot = math.fsum(ws)
        if tot <= 0:
            continue
        p = ws / tot
        nz = p > 0
        if np.any(nz):
            beta = min(beta, float(np.min(ph[a0:a1][nz] / p[nz])))
    return beta


def error_bound(rule, stats, c, beta, delta, blkprod_sq, pilot_sq=None):
    """The bound B with ||MN - CD||_F^2 <= B with probability >= 1 - delta,
    and the bound V on the sum of the asymptotic variances, for Alg. 2 with
    probabilities >= beta (3.8) and
      'opt'      block sizes (3.9): Thm 3.3, (3.11) and (3.12);
      'norm'     block sizes (4.2): Thm 4.2, (4.3) and (4.4);
      'two_step' block sizes (4.7): Thm 4.4, (4.8) and (4.9), with the
                 pilot estimates pilot_sq.
    v_k s_k = ||M^k N_k||_F gives theta_1 <= 1 - v_k^2 <= theta_2 (min and
    max over the blocks with s_k > 0); the pilot's v^_k s_k =
    ||C^{0k} D_{0k}||_F gives theta^_1 <= |1 - v^_k^2| <= theta^_2.
    Returns dict(phi, eta, var_bound, bound, theta1, theta2[, theta1_hat,
    theta2_hat]); phi is infinite when theta_1 = 0 for 'opt'. In (4.8) the
    numerator of phi~ carries theta_2 of Thm 3.3 (the exact v_k) beside the
    pilot's theta^, as printed; its exponent (theta^_2 theta^_1)^(1/4) is read
    as in Thm 3.3."""
    s = np.asarray(stats.s, np.float64)
    live = s > 0
    v2 = np.asarray(blkprod_sq, np.float64)[live] / (s[live] ** 2)
    t1, t2 = float(np.min(1.0 - v2)), float(np.max(1.0 - v2))
    mn = math.fsum(stats.m_sq) * math.fsum(stats.n_sq)
    tail = math.sqrt((8.0 / beta) * math.log(1.0 / delta))
    out = dict(theta1=t1, theta2=t2)
    if rule == "opt":
        phi = (math.sqrt(t2 - t1 * beta + t2 * t1 * beta) / (t2 * t1) ** 0.25
               if t1 > 0 else math.inf)
        eta = phi + (math.sqrt(t2 / t1) * tail if t1 > 0 else math.inf)
    elif rule == "norm":
        phi = math.sqrt(1.0 - beta * (1.0 - t2))
        eta = phi + tail
    elif rule == "two_step":
        vh2 = np.asarray(pilot_sq, np.float64)[live] / (s[live] ** 2)
        h1, h2 = float(np.min(np.abs(1.0 - vh2))), float(np.max(np.abs(1.0 - vh2)))
        out.update(theta1_hat=h1, theta2_hat=h2)
        phi = (math.sqrt(h2 - h1 * beta + t2 * h1 * beta) / (h2 * h1) ** 0.25
               if h1 > 0 else math.inf)
        eta = phi + (math.sqrt(h2 / h1) * tail if h1 > 0 else math.inf)
    else:
        raise ValueError(f"no bound for rule {rule!r}")
    out.update(phi=phi, eta=eta, var_bound=phi * phi / (beta * c) * mn,
               bound=eta * eta / (beta * c) * mn)
    return out


# ----------------------------------------------------------------------------
# Whole pipeline
# ----------------------------------------------------------------------------

@dataclass
class Result:
    design: Design
    draws: Draws
    col_sq: np.ndarray
    row_sq: np.ndarray
    stats: BlockStats
    C: np.ndarray
    D: np.ndarray
    CD: np.ndarray
    MN: np.ndarray
    err: float
    rel: float


def plan(M, N, off, c, mode="block", prob="norm", alloc="norm", user_w=None,
         user_ck=None, blkprod_sq=None, col_row=None, pilot_sq=None):
    """Norms -> weights -> design (everything before the random draws).
    Rule 'two_step' takes the pilot estimates (``pilot``) as pilot_sq."""
    n = M.shape[1]
    off = check_partition(off, n)
    col_sq, row_sq = col_row if col_row is not None else column_row_sq(M, N)
    stats = block_stats(col_sq, row_sq, off)
    need_prod = (prob == "exact") or (mode == "stratified" and alloc == "opt")
    if need_prod and blkprod_sq is None:
        blkprod_sq = block_product_sq(M, N, off)
    w = atom_weights(mode, prob, off, col_sq, row_sq, stats, blkprod_sq, user_w)
    g = None
    if mode == "stratified" and alloc != "user":
        g = alloc_weights(alloc, stats, blkprod_sq, pilot_sq)
    design = make_design(mode, off, c, w, g,
                         user_ck if (mode == "stratified" and alloc == "user") else None)
    return design, col_sq, row_sq, stats


def run(M, N, off, c, seed=0, trial=0, mode="block", prob="norm",
        alloc="norm", user_w=None, user_ck=None, blkprod_sq=None, c0=None,
        pilot_prob="uniform"):
    """The full forward path: Alg. 2 (or the block sampler, or Alg. 3 when
    alloc is 'two_step': the pilot with c0 draws first), its product and the
    judge."""
    pilot_sq = None
    col_row = None
    if mode == "stratified" and alloc == "two_step":
        col_row = column_row_sq(M, N)
        pilot_sq = pilot(M, N, off, c0, pilot_prob, seed, trial, col_row).pilot_sq
    design, col_sq, row_sq, stats = plan(M, N, off, c, mode, prob, alloc,
                                         user_w, user_ck, blkprod_sq, col_row,
                                         pilot_sq)
    draws = sample(design, seed, trial)
    C, D = sketch(M, N, draws)
    CD = sketch_product(C, D)
    MN = exact_product(M, N)
    err, rel, _, _ = judge(MN, CD)
    return Result(design, draws, col_sq, row_sq, stats, C, D, CD, MN, err, rel)


# ----------------------------------------------------------------------------
# Gradient of the sketch
# ----------------------------------------------------------------------------

def backward(M, N, draws, G):
    """Gradients of <G, CD> with respect to M and N, the draws held fixed.

    CD = sum_t scale_t^2 M[:, atom_t] N[atom_t, :] (3.3) is linear in M for
    fixed N and the other way round, so

        dM[:, atom] = (sum of scale_t^2 over draws t of that atom) G N[atom, :]^T
        dN[atom, :] = (same factor) M[:, atom]^T G

    and every column of M (row of N) outside the drawn atoms gets zero.
    """
    M64 = np.asarray(M, np.float64)
    N64 = np.asarray(N, np.float64)
    G64 = np.asarray(G, np.float64)
    dM = np.zeros_like(M64)
    dN = np.zeros_like(N64)
    fac = {}
    for t in range(len(draws.atom)):
        key = (int(draws.lo[t]), int(draws.width[t]))
        fac[key] = fac.get(key, 0.0) + draws.scale[t] ** 2
    for (lo, wd), f in fac.items():
        dM[:, lo:lo + wd] = f * (G64 @ N64[lo:lo + wd, :].T)
        dN[lo:lo + wd, :] = f * (M64[:, lo:lo + wd].T @ G64)
    return dM, dN
