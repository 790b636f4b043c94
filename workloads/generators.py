"""Seeded generators for the synthetic MDP workloads.

Every instance is a discounted-cost MDP in the form the paper's problem setting
uses (finite states S, finite actions A, stage costs g(s, a), discount gamma,
row-stochastic transitions), stored as a CSR matrix with S*A rows, row
r = s*A + a (state-major), S columns, sorted unique int32 column indices and
float64 probabilities.

Randomness: numpy PCG64 streams keyed by SeedSequence([SEED_BASE, cfg, seed,
chunk]).  Large instances are drawn in fixed chunks of states, each from its own
stream, so the result does not depend on how many worker threads run.

Nothing here computes any part of the solution method; the module only draws
and arranges random numbers.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1447402502
GEN_VERSION = 1


@dataclass
class MDPInstance:
    S: int
    A: int
    row_ptr: np.ndarray  # int64, S*A + 1
    col: np.ndarray      # int32, nnz
    val: np.ndarray      # float64, nnz
    cost: np.ndarray     # float64, S*A
    gamma: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def rows(self) -> int:
        return self.S * self.A


def _rng(cfg: int, seed: int, chunk: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE, cfg, seed, chunk]))


def _workers(workers):
    if workers is not None:
        return max(1, int(workers))
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _distinct_sorted(rng, n, k, low, high):
    """n rows of k distinct integers drawn uniformly from [low, high), each row sorted.

    Whole rows with a repeated value are redrawn, which gives the uniform law
    over k-subsets."""
    out = rng.integers(low, high, size=(n, k), dtype=np.int64)
    out.sort(axis=1)
    bad = np.any(out[:, 1:] == out[:, :-1], axis=1) if k > 1 else np.zeros(n, bool)
    while bad.any():
        idx = np.nonzero(bad)[0]
        redo = rng.integers(low, high, size=(idx.size, k), dtype=np.int64)
        redo.sort(axis=1)
        out[idx] = redo
        sub_bad = np.any(redo[:, 1:] == redo[:, :-1], axis=1)
        bad = np.zeros(n, bool)
        bad[idx[sub_bad]] = True
    return out


def _band_plus_jumps(rng, srow, S, n_band, n_jump, halfwidth):
    """Columns for rows whose state index is srow: n_band distinct offsets from
    [-halfwidth, halfwidth] taken mod S, plus n_jump uniform columns in [0, S);
    the jumps are redrawn until all n_band + n_jump columns of a row differ.
    Returns sorted columns, shape (len(srow), n_band + n_jump)."""
    n = srow.shape[0]
    if n_band > 0:
        off = _distinct_sorted(rng, n, n_band, -halfwidth, halfwidth + 1)
        band = (srow[:, None] + off) % S
    else:
        band = np.empty((n, 0), np.int64)
    if n_jump == 0:
        cols = np.sort(band, axis=1)
        return cols
    jumps = rng.integers(0, S, size=(n, n_jump), dtype=np.int64)
    cols = np.concatenate([band, jumps], axis=1)
    cols.sort(axis=1)
    bad = np.any(cols[:, 1:] == cols[:, :-1], axis=1)
    while bad.any():
        idx = np.nonzero(bad)[0]
        j2 = rng.integers(0, S, size=(idx.size, n_jump), dtype=np.int64)
        c2 = np.concatenate([band[idx], j2], axis=1)
        c2.sort(axis=1)
        cols[idx] = c2
        sub_bad = np.any(c2[:, 1:] == c2[:, :-1], axis=1)
        bad = np.zeros(n, bool)
        bad[idx[sub_bad]] = True
    return cols


def _normalise_rows(w):
    return w / w.sum(axis=1, keepdims=True)


def _assemble_fixed_k(S, A, k, chunk_fn, n_chunks, chunk_states, workers):
    """Run chunk_fn(chunk_index) -> (cols (n,k), vals (n,k), cost (n,)) over all
    chunks and pack the results into CSR arrays with exactly k entries per row."""
    rows = S * A
    nnz = rows * k
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    cost = np.empty(rows, np.float64)

    def run(c):
        s0 = c * chunk_states
        s1 = min(S, s0 + chunk_states)
        cc, vv, gg = chunk_fn(c, s0, s1)
        r0, r1 = s0 * A, s1 * A
        col[r0 * k:r1 * k] = cc.reshape(-1)
        val[r0 * k:r1 * k] = vv.reshape(-1)
        cost[r0:r1] = gg

    nw = _workers(workers)
    if nw == 1 or n_chunks == 1:
        for c in range(n_chunks):
            run(c)
    else:
        with ThreadPoolExecutor(nw) as ex:
            list(ex.map(run, range(n_chunks)))
    row_ptr = np.arange(rows + 1, dtype=np.int64) * k
    return row_ptr, col, val, cost


def config1(S=1000, A=4, k=10, gamma=0.9, seed=0):
    """Uniform random sparse MDP: k columns per row drawn uniformly without
    replacement, Uniform(0,1) weights normalised to sum 1, Uniform(0,1) costs."""
    if k > S:
        raise ValueError("k > S")
    rng = _rng(1, seed, 0)
    rows = S * A
    cols = _distinct_sorted(rng, rows, k, 0, S)
    w = rng.random((rows, k))
    vals = _normalise_rows(w)
    cost = rng.random(rows)
    row_ptr = np.arange(rows + 1, dtype=np.int64) * k
    return MDPInstance(S, A, row_ptr, cols.astype(np.int32).reshape(-1), vals.reshape(-1), cost,
                       float(gamma), name="uniform-random",
                       meta=dict(cfg=1, seed=seed, k=k, gen_version=GEN_VERSION))


def config2(S=1_000_000, A=8, n_band=14, n_jump=2, halfwidth=64, gamma=0.99, seed=0,
            chunk_states=65536, workers=None):
    """Banded-plus-long-jump MDP: per row, n_band distinct columns within
    +-halfwidth of s (mod S) and n_jump uniform long jumps, all distinct;
    probabilities from Dirichlet(1); Uniform(0,1) costs."""
    k = n_band + n_jump
    if S <= 2 * halfwidth + 1 + n_jump:
        raise ValueError("S too small for the band")
    n_chunks = (S + chunk_states - 1) // chunk_states

    def chunk(c, s0, s1):
        rng = _rng(2, seed, c)
        srow = np.repeat(np.arange(s0, s1, dtype=np.int64), A)
        cols = _band_plus_jumps(rng, srow, S, n_band, n_jump, halfwidth)
        vals = _normalise_rows(rng.standard_exponential((srow.size, k)))
        cost = rng.random(srow.size)
        return cols, vals, cost

    row_ptr, col, val, cost = _assemble_fixed_k(S, A, k, chunk, n_chunks, chunk_states, workers)
    return MDPInstance(S, A, row_ptr, col, val, cost, float(gamma), name="band-jump-dirichlet1",
                       meta=dict(cfg=2, seed=seed, k=k, gen_version=GEN_VERSION))


MAZE_ACTIONS = ("stay", "N", "S", "E", "W")


def config3(H=2000, W=2000, p_move=0.8, obstacle_frac=0.2, gamma=0.999, seed=0,
            chunk_states=262144, workers=None):
    """Grid maze.  State s = i*W + j.  Actions 0 stay, 1 N (i-1), 2 S (i+1),
    3 E (j+1), 4 W (j-1).  The chosen action's target is reached with
    probability p_move; each of the four other actions' targets with
    (1 - p_move)/4.  Moves off the grid stay put.  Obstacles are i.i.d. cells
    (cost 10, absorbing); the goal (H-1, W-1) is forced free (cost 0, absorbing);
    every other cell costs 1 for every action.  Targets that coincide are merged
    into one entry holding the summed probability."""
    S = H * W
    A = 5
    rng0 = _rng(3, seed, 0)
    obstacle = rng0.random(S) < obstacle_frac
    goal = S - 1
    obstacle[goal] = False
    absorbing = obstacle.copy()
    absorbing[goal] = True
    p_slip = (1.0 - p_move) / 4.0
    n_chunks = (S + chunk_states - 1) // chunk_states

    parts = [None] * n_chunks

    def chunk(c):
        s0 = c * chunk_states
        s1 = min(S, s0 + chunk_states)
        s = np.arange(s0, s1, dtype=np.int64)
        i, j = s // W, s % W
        tgt = np.stack([
            s,
            np.where(i > 0, s - W, s),
            np.where(i < H - 1, s + W, s),
            np.where(j < W - 1, s + 1, s),
            np.where(j > 0, s - 1, s),
        ], axis=1)                                   # (ns, 5) target of each action
        ns = s.size
        absb = absorbing[s0:s1]
        tgt[absb] = s[absb, None]
        cols5 = np.repeat(tgt, A, axis=0)            # (ns*A, 5): row (s, a)
        a_of_row = np.tile(np.arange(A), ns)
        p5 = np.where(np.arange(5)[None, :] == a_of_row[:, None], p_move, p_slip)
        order = np.argsort(cols5, axis=1, kind="stable")
        cs = np.take_along_axis(cols5, order, axis=1)
        ps = np.take_along_axis(p5, order, axis=1)
        first = np.ones_like(cs, dtype=bool)
        first[:, 1:] = cs[:, 1:] != cs[:, :-1]
        flat_first = first.reshape(-1)
        gid = np.cumsum(flat_first) - 1
        mval = np.bincount(gid, weights=ps.reshape(-1))
        mcol = cs.reshape(-1)[flat_first]
        counts = first.sum(axis=1)
        row_absorbing = np.repeat(absb, A)
        starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
        mval[starts[row_absorbing]] = 1.0
        cost = np.where(np.repeat(obstacle[s0:s1], A), 10.0, 1.0)
        cost[np.repeat(s == goal, A)] = 0.0
        parts[c] = (counts, mcol.astype(np.int32), mval, cost)

    nw = _workers(workers)
    if nw == 1 or n_chunks == 1:
        for c in range(n_chunks):
            chunk(c)
    else:
        with ThreadPoolExecutor(nw) as ex:
            list(ex.map(chunk, range(n_chunks)))
    counts = np.concatenate([p[0] for p in parts])
    row_ptr = np.zeros(S * A + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.concatenate([p[1] for p in parts])
    val = np.concatenate([p[2] for p in parts])
    cost = np.concatenate([p[3] for p in parts])
    return MDPInstance(S, A, row_ptr, col, val, cost, float(gamma), name="grid-maze",
                       meta=dict(cfg=3, seed=seed, H=H, W=W, obstacle=obstacle, goal=goal,
                                 gen_version=GEN_VERSION))


def config4(S=4_000_000, A=16, k=24, alpha=0.5, gamma=0.995, seed=0, chunk_states=32768,
            workers=None):
    """Uniform random columns (k per row, without replacement), Dirichlet(alpha)
    probabilities (normalised Gamma(alpha) draws) and Lognormal(0,1) costs."""
    if k > S:
        raise ValueError("k > S")
    n_chunks = (S + chunk_states - 1) // chunk_states

    def chunk(c, s0, s1):
        rng = _rng(4, seed, c)
        n = (s1 - s0) * A
        cols = _distinct_sorted(rng, n, k, 0, S)
        vals = _normalise_rows(rng.gamma(alpha, size=(n, k)))
        cost = rng.lognormal(0.0, 1.0, size=n)
        return cols, vals, cost

    row_ptr, col, val, cost = _assemble_fixed_k(S, A, k, chunk, n_chunks, chunk_states, workers)
    return MDPInstance(S, A, row_ptr, col, val, cost, float(gamma), name="uniform-dirichlet0.5",
                       meta=dict(cfg=4, seed=seed, k=k, gen_version=GEN_VERSION))


GAMMAS5 = (0.9, 0.99, 0.999)


def config5_requests(n=10000, seed=0, s_min_exp=3.0, s_max_exp=6.0):
    """The request stream of the serving load: per request S = round(10**U),
    A uniform in {2..16}, k uniform in {4..32}, gamma uniform over {0.9, 0.99,
    0.999}, a per-request instance seed and a unit-rate exponential
    inter-arrival gap (scaled by 1/lambda by the caller)."""
    rng = _rng(5, seed, 0)
    S = np.rint(10.0 ** rng.uniform(s_min_exp, s_max_exp, size=n)).astype(np.int64)
    A = rng.integers(2, 17, size=n)
    k = rng.integers(4, 33, size=n)
    g = np.asarray(GAMMAS5)[rng.integers(0, 3, size=n)]
    gaps = rng.standard_exponential(n)
    return [dict(id=i, S=int(S[i]), A=int(A[i]), k=int(k[i]), gamma=float(g[i]),
                 gap=float(gaps[i]), seed=int(seed) * 1_000_003 + i) for i in range(n)]


def config5_instance(req, halfwidth=64, chunk_states=65536, workers=1):
    """One serving request: ceil(k/2) distinct band columns within +-halfwidth
    of s (mod S) plus floor(k/2) uniform long jumps, all distinct; Dirichlet(1)
    probabilities; Uniform(0,1) costs."""
    S, A, k = req["S"], req["A"], req["k"]
    n_band = (k + 1) // 2
    n_jump = k // 2
    if S <= 2 * halfwidth + 1 + n_jump:
        raise ValueError("S too small for the band")
    n_chunks = (S + chunk_states - 1) // chunk_states

    def chunk(c, s0, s1):
        rng = _rng(5, req["seed"] + 1, c)
        srow = np.repeat(np.arange(s0, s1, dtype=np.int64), A)
        cols = _band_plus_jumps(rng, srow, S, n_band, n_jump, halfwidth)
        vals = _normalise_rows(rng.standard_exponential((srow.size, k)))
        cost = rng.random(srow.size)
        return cols, vals, cost

    row_ptr, col, val, cost = _assemble_fixed_k(S, A, k, chunk, n_chunks, chunk_states, workers)
    return MDPInstance(S, A, row_ptr, col, val, cost, req["gamma"], name="serve-request",
                       meta=dict(cfg=5, req=dict(req), k=k, gen_version=GEN_VERSION))


def random_dense_mdp(S, A, gamma, seed=0, density=1.0, cost_scale=1.0):
    """Small random MDP with a random sparsity pattern (each row keeps every
    column with probability `density`, at least one), Uniform(0,1) weights and
    costs.  For tests at small S."""
    rng = _rng(100, seed, S * 1000 + A)
    rows = S * A
    keep = rng.random((rows, S)) < density
    force = rng.integers(0, S, size=rows)
    keep[np.arange(rows), force] = True
    w = rng.random((rows, S)) * keep
    w[np.arange(rows), force] += 0.5
    dense = w / w.sum(axis=1, keepdims=True)
    counts = keep.sum(axis=1)
    row_ptr = np.zeros(rows + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    rr, cc = np.nonzero(keep)
    col = cc.astype(np.int32)
    val = dense[rr, cc]
    cost = rng.random(rows) * cost_scale
    return MDPInstance(S, A, row_ptr, col, val, cost, float(gamma), name="random-small",
                       meta=dict(cfg=100, seed=seed, density=density))


def deterministic_chain(n, c_adv=1.0, c_stay=2.0, gamma=0.9):
    """Chain of n states with two actions.  Action 0 (advance) costs c_adv and
    moves s -> s+1; action 1 (stay) costs c_stay and stays.  State n-1 is
    absorbing with cost 0 under both actions."""
    A = 2
    rows = n * A
    col = np.empty(rows, np.int32)
    cost = np.empty(rows, np.float64)
    for s in range(n):
        if s == n - 1:
            col[2 * s] = s
            col[2 * s + 1] = s
            cost[2 * s] = 0.0
            cost[2 * s + 1] = 0.0
        else:
            col[2 * s] = s + 1
            col[2 * s + 1] = s
            cost[2 * s] = c_adv
            cost[2 * s + 1] = c_stay
    row_ptr = np.arange(rows + 1, dtype=np.int64)
    val = np.ones(rows, np.float64)
    return MDPInstance(n, A, row_ptr, col, val, cost, float(gamma), name="chain",
                       meta=dict(c_adv=c_adv, c_stay=c_stay))


def describe(inst: MDPInstance) -> dict:
    return dict(name=inst.name, S=inst.S, A=inst.A, nnz=inst.nnz, gamma=inst.gamma,
                k_mean=inst.nnz / max(1, inst.rows),
                **{k: v for k, v in inst.meta.items() if isinstance(v, (int, float, str))})
