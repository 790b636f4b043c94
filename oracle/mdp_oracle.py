"""Plain float64 CPU reference for discounted-cost MDPs (test infrastructure).

Notation (the paper's problem setting): S states, A actions, stage cost
g(s, a), discount gamma in [0, 1), transition probabilities P[(s, a), s'].  Row
r = s*A + a of the CSR matrix holds P[(s, a), :].

    Q_v(s, a)  = g(s, a) + gamma * sum_j P[(s, a), j] v_j
    (T v)(s)   = min_a Q_v(s, a)               (Bellman operator, minimisation)
    pi_v(s)    = lowest a attaining the minimum (greedy policy)
    T_pi v     = g_pi + gamma P_pi v,  P_pi[s, :] = P[(s, pi(s)), :]

The optimal value v* is the unique fixed point of T (T is a gamma-contraction
in the max norm).  Exact policy iteration alternates greedy improvement with an
exact solve of (I - gamma P_pi) v = g_pi and reaches v* in finitely many steps;
that is the result the inexact method of the paper approximates ("Problem
Setting and Solution Methods" section).

Nothing here is blocked, fused or reordered: each step is the definition
written out, with scipy/numpy primitives (sparse matvec, LU solve) as steps.
"""
from __future__ import annotations

import itertools

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

DENSE_MAX_S = 2500


def to_csr(inst):
    """The S*A x S transition matrix as a scipy CSR matrix (float64)."""
    return sp.csr_matrix((inst.val, inst.col.astype(np.int64), inst.row_ptr),
                         shape=(inst.S * inst.A, inst.S))


def q_values(inst, v, P=None):
    """Q_v(s, a) = g(s, a) + gamma * (P v)(s, a), shape (S, A)."""
    P = to_csr(inst) if P is None else P
    v = np.asarray(v, np.float64)
    return (inst.cost + inst.gamma * (P @ v)).reshape(inst.S, inst.A)


def q_values_states(inst, v, states):
    """Q_v(s, a) for the given states only, shape (len(states), A): each row's
    sum over its stored entries, taken straight from the CSR arrays.  For
    spot checks on instances too large to handle whole."""
    v = np.asarray(v, np.float64)
    states = np.asarray(states, np.int64)
    Q = np.empty((states.size, inst.A))
    for i, s in enumerate(states):
        for a in range(inst.A):
            r = s * inst.A + a
            lo, hi = inst.row_ptr[r], inst.row_ptr[r + 1]
            Q[i, a] = inst.cost[r] + inst.gamma * np.dot(inst.val[lo:hi], v[inst.col[lo:hi]])
    return Q


def bellman(inst, v, P=None):
    """One Bellman sweep: (T v, greedy policy, ||T v - v||_inf).

    numpy's argmin returns the first minimiser, i.e. the lowest action index
    on exact ties."""
    Q = q_values(inst, v, P)
    Tv = Q.min(axis=1)
    pi = Q.argmin(axis=1).astype(np.int32)
    res = float(np.max(np.abs(Tv - np.asarray(v, np.float64)))) if inst.S else 0.0
    return Tv, pi, res


def bellman_streamed(inst, v, block_rows=1 << 22, workers=1):
    """The same sweep as bellman() (the problem statement's Bellman operator:
    minimum over actions of cost plus discounted expected value), computed
    straight from the CSR arrays a block of rows at a time, so that matrices
    with billions of stored entries need no scipy copy.  Blocks are
    independent; `workers` threads may take them.  Returns
    (T v, greedy policy, ||T v - v||_inf)."""
    v = np.asarray(v, np.float64)
    rows = inst.S * inst.A
    Q = np.empty(rows)

    def block(r0):
        r1 = min(rows, r0 + block_rows)
        lo, hi = int(inst.row_ptr[r0]), int(inst.row_ptr[r1])
        if np.any(np.diff(inst.row_ptr[r0:r1 + 1]) <= 0):
            raise ValueError("empty row")
        terms = inst.val[lo:hi] * v[inst.col[lo:hi]]
        starts = (inst.row_ptr[r0:r1] - lo).astype(np.int64)
        Q[r0:r1] = inst.cost[r0:r1] + inst.gamma * np.add.reduceat(terms, starts)

    starts = range(0, rows, block_rows)
    if workers > 1:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(block, starts))
    else:
        for r0 in starts:
            block(r0)
    Q = Q.reshape(inst.S, inst.A)
    Tv = Q.min(axis=1)
    pi = Q.argmin(axis=1).astype(np.int32)
    res = float(np.max(np.abs(Tv - v))) if inst.S else 0.0
    return Tv, pi, res


def policy_system(inst, pi, P=None):
    """(P_pi as S x S CSR, g_pi): the rows s*A + pi(s) of P and of g."""
    P = to_csr(inst) if P is None else P
    rows = np.arange(inst.S, dtype=np.int64) * inst.A + np.asarray(pi, np.int64)
    return P[rows], inst.cost[rows]


def _true_residual(M, b, v):
    return float(np.max(np.abs(b - M @ v))) if v.size else 0.0


def evaluate_policy(inst, pi, P=None, method="auto", tol=1e-12):
    """v_pi, the exact solution of (I - gamma P_pi) v = g_pi.

    method: "dense" (LAPACK LU), "sparse" (SuperLU) or "certified"
    (restarted GMRES plus iterative refinement until the true residual r
    certifies the error: ||v - v_pi||_inf <= ||r||_inf / (1 - gamma)
    <= tol * max(1, ||v||_inf)).
    "auto" picks dense for S <= DENSE_MAX_S and the certified mode otherwise
    (sparse LU fills in badly on random long-range columns).
    Returns (v, true residual in the max norm)."""
    Ppi, gpi = policy_system(inst, pi, P)
    S = inst.S
    M = (sp.identity(S, format="csr") - inst.gamma * Ppi).tocsr()
    if method == "auto":
        method = "dense" if S <= DENSE_MAX_S else "certified"
    if method == "dense":
        v = scipy.linalg.solve(M.toarray(), gpi)
    elif method == "sparse":
        v = spla.spsolve(M.tocsc(), gpi)
    elif method == "certified":
        v = np.zeros(S)
        for _ in range(100):
            r = gpi - M @ v
            if np.max(np.abs(r)) / (1.0 - inst.gamma) <= tol * max(1.0, np.max(np.abs(v))):
                break
            d, info = spla.gmres(M, r, rtol=1e-12, atol=0.0, restart=100, maxiter=100)
            v = v + d
        else:
            raise RuntimeError("certified policy evaluation did not reach its residual bound")
    else:
        raise ValueError(method)
    v = np.asarray(v, np.float64)
    return v, _true_residual(M, gpi, v)


def policy_iteration(inst, v0=None, tol=1e-10, max_iter=500, method="auto", check_monotone=True):
    """Exact policy iteration.

    From v_0 (zero unless given): sweep to get the greedy policy pi_k and
    res_k = ||T v_k - v_k||_inf; stop when res_k <= tol or the policy repeats;
    else v_{k+1} = v_{pi_k} by an exact solve.  Evaluated values decrease
    monotonically (T_{pi_k} v_k = T v_k <= v_k for k >= 1 and T_pi is monotone).
    Returns dict(v, pi, res, iters, history)."""
    P = to_csr(inst)
    v = np.zeros(inst.S) if v0 is None else np.asarray(v0, np.float64).copy()
    hist = []
    prev_pi = None
    for k in range(max_iter + 1):
        Tv, pi, res = bellman(inst, v, P)
        hist.append(res)
        if res <= tol or (prev_pi is not None and np.array_equal(pi, prev_pi)):
            return dict(v=v, pi=pi, res=res, iters=k, history=hist)
        if k == max_iter:
            break
        v_new, _ = evaluate_policy(inst, pi, P, method=method)
        if check_monotone and k >= 1:
            slack = 1e-11 * max(1.0, float(np.max(np.abs(v))))
            if np.any(v_new > v + slack):
                raise AssertionError("policy iteration lost monotonicity")
        v = v_new
        prev_pi = pi
    return dict(v=v, pi=pi, res=res, iters=max_iter, history=hist)


def evaluate_policy_fixed_point(inst, pi, P=None, tol=1e-14, max_iter=1_000_000):
    """v_pi by repeating v <- T_pi v from v = 0 until successive iterates differ
    by at most tol * max(1, ||v||_inf) times (1 - gamma) / gamma.  The error
    is then below tol * max(1, ||v||_inf) (contraction bound).  Uses no linear
    solve, so it is independent of evaluate_policy."""
    Ppi, gpi = policy_system(inst, pi, P)
    v = np.zeros(inst.S)
    g = inst.gamma
    for _ in range(max_iter):
        nv = gpi + g * (Ppi @ v)
        d = float(np.max(np.abs(nv - v)))
        v = nv
        if g == 0.0 or d <= tol * max(1.0, float(np.max(np.abs(v)))) * (1.0 - g) / g:
            return v
    raise RuntimeError("fixed-point evaluation did not converge")


def brute_force(inst, maximize=False):
    """v* as the elementwise minimum (maximize=True: maximum, with inst.cost
    read as rewards) of v_pi over all A**S deterministic policies (each
    evaluated by fixed-point iteration), and every (policy, v_pi) pair.
    For S*log(A) small only."""
    P = to_csr(inst)
    best = None
    vals = []
    pick = np.maximum if maximize else np.minimum
    for pol in itertools.product(range(inst.A), repeat=inst.S):
        pi = np.asarray(pol, np.int32)
        v = evaluate_policy_fixed_point(inst, pi, P)
        vals.append((pi, v))
        best = v.copy() if best is None else pick(best, v)
    return best, vals


def macqueen_bounds(inst, v, P=None):
    """MacQueen's componentwise bounds on v* from any v:
        T v + gamma/(1-gamma) * min(T v - v) <= v* <= T v + gamma/(1-gamma) * max(T v - v)."""
    Tv, _, _ = bellman(inst, v, P)
    d = Tv - np.asarray(v, np.float64)
    c = inst.gamma / (1.0 - inst.gamma)
    return Tv + c * d.min(), Tv + c * d.max()


def value_iteration(inst, v0=None, tol=1e-10, max_iter=100000):
    """v <- T v until ||T v - v||_inf <= tol; returns (v, pi, res, iters) with
    pi greedy for the returned v (the same return convention as policy
    iteration)."""
    P = to_csr(inst)
    v = np.zeros(inst.S) if v0 is None else np.asarray(v0, np.float64).copy()
    for k in range(max_iter + 1):
        Tv, pi, res = bellman(inst, v, P)
        if res <= tol or k == max_iter:
            return v, pi, res, k
        v = Tv


def modified_policy_iteration(inst, m, v0=None, tol=1e-10, max_iter=100000):
    """Modified policy iteration: greedy sweep, then m applications of
    T_pi starting from v (the first one equals T v)."""
    P = to_csr(inst)
    v = np.zeros(inst.S) if v0 is None else np.asarray(v0, np.float64).copy()
    for k in range(max_iter + 1):
        Tv, pi, res = bellman(inst, v, P)
        if res <= tol or k == max_iter:
            return v, pi, res, k
        Ppi, gpi = policy_system(inst, pi, P)
        x = v
        for _ in range(m):
            x = gpi + inst.gamma * (Ppi @ x)
        v = x


def fp16_with_row_correction(inst):
    """Half-precision copy of P with a per-row float64 correction
    c_r = 1 - sum_j float64(fp16(p_rj)) (round-to-nearest-even conversion)."""
    h = inst.val.astype(np.float16)
    hs = h.astype(np.float64)
    rows = inst.S * inst.A
    c = np.empty(rows)
    for r in range(rows):
        c[r] = 1.0 - hs[inst.row_ptr[r]:inst.row_ptr[r + 1]].sum()
    return h, c


def policy_parity(inst, q_star, pi_hat, pi_star, tau):
    """Policy comparison rule: where the oracle's action-value gap (second
    smallest minus smallest Q*) exceeds tau the actions must agree; everywhere
    the chosen action must be tau-optimal.  Returns a dict of counts."""
    S, A = q_star.shape
    qmin = q_star.min(axis=1)
    if A > 1:
        part = np.partition(q_star, 1, axis=1)
        gap = part[:, 1] - part[:, 0]
    else:
        gap = np.full(S, np.inf)
    chosen = q_star[np.arange(S), pi_hat]
    strict = gap > tau
    return dict(
        mismatch_outside_band=int(np.sum(strict & (pi_hat != pi_star))),
        not_tau_optimal=int(np.sum(chosen - qmin > tau)),
        ties_1e9=int(np.sum(gap <= 1e-9)),
        excused=int(np.sum((gap > 1e-9) & (gap <= tau))),
    )
