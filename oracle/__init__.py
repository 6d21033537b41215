"""CPU oracle for the D-iteration PageRank solve -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct fp64 implementations written from the paper
("Optimized on-line computation of PageRank algorithm", arXiv 1202.6158):

* :func:`dense_exact` -- the plain definition of the limit, Y = (1-d)(I-dP)^{-1}V
  (Section 2.2: S_inf = X), by LU on the dense matrix; ``x* = Y/||Y||_1``
  (Section 3.3: renormalisation when P has dangling columns).
* :func:`completed_pagerank` -- the stationary vector of the completed matrix
  A = d Pbar + (1-d) V 1^t, whose zero columns are replaced by V (Section 2.1),
  by eigen-decomposition; Section 3.3 states it equals ``x*``.
* :func:`sparse_exact` -- the same definition by a sparse direct solve.
* :func:`diter` -- the sequential D-iteration (ALGO-REF with the dangling rule,
  Sections 2.2 and 3.3) in the orders of Section 4 (PER, RAND, MAX, threshold
  sweeps, OP, OP2), in C.
* :func:`set_step` / :func:`diter_sets` -- diffusion of a whole threshold set at
  once (J_{i_n} replaced by the selector of a set), in C.
* :func:`power` -- MAT-ITER X_{n+1} = dPX_n + (1-d)V from X_0 = 0 (Sections 2.1, 4),
  in C.
* :func:`inject_update` -- the fluid a graph update injects, F' = F + d(P'-P)H
  (updating equation, Section 3.2); :func:`set_step_signed` -- a set step on
  fluid of either sign (|F_i| against the threshold), in numpy.
* :func:`dense_exact_weighted` / :func:`set_step_weighted` -- the limit and a set
  step for a weighted P (any column-stochastic P of Section 2.1), in numpy.
* :func:`apply_set` -- diffusion of a given set, for replaying the sets a solve
  recorded round by round, in numpy.
* :func:`limit` -- ``x*`` by :func:`dense_exact` on small graphs, else by
  :func:`power` run to a tolerance far below the one under test.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "diter.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib_handle = None

PER, RAND, MAX, SWEEP, OP, OP2 = 0, 1, 2, 3, 4, 5
ORDERS = {"per": PER, "rand": RAND, "max": MAX, "sweep": SWEEP, "op": OP, "op2": OP2}


class Stats(ctypes.Structure):
    _fields_ = [("picks", ctypes.c_int64), ("edges", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("residual", ctypes.c_double),
                ("running_r", ctypes.c_double), ("converged", ctypes.c_int32),
                ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


def build(force: bool = True) -> str:
    """Compile oracle/diter.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", "-o",
                               tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        p, i64, dbl, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(Stats)
        lib.or_diter.restype = ctypes.c_int
        lib.or_diter.argtypes = [i64, p, p, dbl, dbl, ctypes.c_int, dbl, ctypes.c_uint64,
                                 i64, dbl, p, p, p, i64, st]
        lib.or_set_step.restype = i64
        lib.or_set_step.argtypes = [i64, p, p, dbl, dbl, p, p, p, st]
        lib.or_diter_sets.restype = ctypes.c_int
        lib.or_diter_sets.argtypes = [i64, p, p, dbl, dbl, dbl, i64, dbl, p, p, st]
        lib.or_power.restype = ctypes.c_int
        lib.or_power.argtypes = [i64, p, p, p, dbl, dbl, i64, p, st]
        lib.or_power_omp.restype = ctypes.c_int
        lib.or_power_omp.argtypes = [i64, p, p, p, dbl, dbl, i64, p, st, p]
        _lib_handle = lib
    return _lib_handle


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    return int(g.n), rp, ci


def _v(n, v):
    return np.full(n, 1.0 / n) if v is None else np.ascontiguousarray(v, dtype=np.float64)


# ----------------------------------------------------------------- definition

def transition_dense(g) -> np.ndarray:
    """Dense P with P[j, i] = (#links i->j) / outdeg(i); dangling columns are zero
    (Section 2.1, no completion)."""
    n, rp, ci = _csr(g)
    P = np.zeros((n, n))
    for i in range(n):
        deg = rp[i + 1] - rp[i]
        for e in range(rp[i], rp[i + 1]):
            P[ci[e], i] += 1.0 / deg
    return P


def dense_exact(g, d: float, v=None):
    """(Y, x*) with Y = (1-d)(I - dP)^{-1} V solved by LU, x* = Y / ||Y||_1.
    Y is the limit of H (Section 2.2, S_inf = X; Section 3.1, H_inf = X)."""
    n = int(g.n)
    v = _v(n, v)
    P = transition_dense(g)
    Y = np.linalg.solve(np.eye(n) - d * P, (1.0 - d) * v)
    return Y, Y / np.abs(Y).sum()


def completed_pagerank(g, d: float, v=None) -> np.ndarray:
    """Stationary vector of A = d Pbar + (1-d) V 1^t where Pbar replaces every zero
    column of P by V (Section 2.1), from the eigenvector of eigenvalue 1."""
    n = int(g.n)
    v = _v(n, v)
    Pbar = transition_dense(g)
    dang = Pbar.sum(axis=0) == 0.0
    Pbar[:, dang] = v[:, None]
    A = d * Pbar + (1.0 - d) * np.outer(v, np.ones(n))
    w, vecs = np.linalg.eig(A)
    k = int(np.argmin(np.abs(w - 1.0)))
    x = np.real(vecs[:, k])
    return x / x.sum()


def sparse_exact(g, d: float, v=None):
    """(Y, x*) as dense_exact, by a sparse direct solve (medium sizes)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n, rp, ci = _csr(g)
    v = _v(n, v)
    deg = np.diff(rp)
    src = np.repeat(np.arange(n), deg)
    P = sp.csc_matrix((1.0 / deg[src], (ci.astype(np.int64), src)), shape=(n, n))
    M = (sp.identity(n, format="csc") - d * P).tocsc()
    Y = spla.spsolve(M, (1.0 - d) * v)
    return Y, Y / np.abs(Y).sum()


# ------------------------------------------------------------- the algorithm

def init_state(n: int, d: float, v=None):
    """F_0 = (1-d)V, H_0 = 0 (Section 2.2)."""
    return (1.0 - d) * _v(n, v), np.zeros(n)


def diter(g, d: float, tol: float, order="per", v=None, c: float = 1.0, seed: int = 0,
          max_picks: int = 1 << 62, state=None, trace_len: int = 0):
    """Sequential D-iteration until ||F||_1 < tol.  Returns dict with H, F,
    x = (H+F)/||H+F||_1, stats, and (if trace_len) the ||F||_1 trace."""
    n, rp, ci = _csr(g)
    if state is None:
        F, H = init_state(n, d, v)
        r0 = float(F.sum())
    else:
        F = np.array(state[0], dtype=np.float64)
        H = np.array(state[1], dtype=np.float64)
        r0 = float(F.sum())
    trace = np.zeros(max(trace_len, 1))
    st = Stats()
    rc = _lib().or_diter(n, rp.ctypes.data, ci.ctypes.data, d, tol, ORDERS.get(order, order),
                         c, seed, max_picks, r0, F.ctypes.data, H.ctypes.data,
                         trace.ctypes.data if trace_len else None, trace_len,
                         ctypes.byref(st))
    y = H + F
    out = dict(H=H, F=F, x=y / y.sum(), converged=rc == 0, stats=st.as_dict())
    if trace_len:
        out["trace"] = trace[:min(trace_len, st.picks)]
    return out


def set_step(g, d: float, theta: float, F, H):
    """One set step from state (F, H) with threshold theta.  Returns
    (F', H', taken mask, stats)."""
    n, rp, ci = _csr(g)
    F = np.array(F, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    taken = np.zeros(n, dtype=np.uint8)
    st = Stats()
    _lib().or_set_step(n, rp.ctypes.data, ci.ctypes.data, d, theta, F.ctypes.data,
                       H.ctypes.data, taken.ctypes.data, ctypes.byref(st))
    return F, H, taken.astype(bool), st.as_dict()


def diter_sets(g, d: float, tol: float, c: float = 1.0, v=None, max_rounds: int = 1 << 40,
               state=None):
    """D-iteration by threshold set steps (theta_r = c ||F_r||_1 / N)."""
    n, rp, ci = _csr(g)
    if state is None:
        F, H = init_state(n, d, v)
    else:
        F = np.array(state[0], dtype=np.float64)
        H = np.array(state[1], dtype=np.float64)
    st = Stats()
    rc = _lib().or_diter_sets(n, rp.ctypes.data, ci.ctypes.data, d, tol, c, max_rounds,
                              float(F.sum()), F.ctypes.data, H.ctypes.data, ctypes.byref(st))
    y = H + F
    return dict(H=H, F=F, x=y / y.sum(), converged=rc == 0, stats=st.as_dict())


def power(g, d: float, tol: float, v=None, max_iter: int = 1 << 30):
    """MAT-ITER from X_0 = 0 until ||X_n - X_{n-1}||_1 < tol.  Returns dict with
    X (last iterate), x = X/||X||_1 and stats."""
    n, rp, ci = _csr(g)
    v = _v(n, v)
    X = np.zeros(n)
    st = Stats()
    rc = _lib().or_power(n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, d, tol, max_iter,
                         X.ctypes.data, ctypes.byref(st))
    return dict(X=X, x=X / X.sum(), converged=rc == 0, stats=st.as_dict())


def power_omp(g, d: float, tol: float, v=None, max_iter: int = 1 << 30):
    """MAT-ITER as :func:`power`, computed on every host core (OpenMP pull over
    in-links; only the summation order differs).  The dict also holds the
    thread count used."""
    n, rp, ci = _csr(g)
    v = _v(n, v)
    X = np.zeros(n)
    st = Stats()
    nt = ctypes.c_int32(0)
    rc = _lib().or_power_omp(n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, d, tol, max_iter,
                             X.ctypes.data, ctypes.byref(st), ctypes.byref(nt))
    return dict(X=X, x=X / X.sum(), converged=rc == 0, stats=st.as_dict(), threads=nt.value)


def limit(g, d: float, v=None, tol: float = 1e-14):
    """x* for graphs of any size: dense LU up to 2000 nodes, else MAT-ITER run
    until ||X_n - X_{n-1}||_1 < tol (error <= d tol/(1-d) before normalising)."""
    if g.n <= 2000:
        return dense_exact(g, d, v)[1]
    return power(g, d, tol, v)["x"]


# ------------------------------------------------------------ graph updates

def transition_sparse(g):
    """Sparse P (CSC) with P[j, i] = (#links i->j) / outdeg(i); dangling columns
    are zero (Section 2.1)."""
    import scipy.sparse as sp
    n, rp, ci = _csr(g)
    deg = np.diff(rp)
    src = np.repeat(np.arange(n), deg)
    return sp.csc_matrix((1.0 / deg[src], (ci.astype(np.int64), src)), shape=(n, n))


def inject_update(g_old, g_new, d: float, F, H):
    """Updating equation (Section 3.2): when P becomes P' with the state (F, H)
    of a D-iteration on P, the D-iteration continues on P' from
    F' = F + d (P' - P) H (Theorem 4: H + F' = F_0 + d P' H).  fp64."""
    H = np.asarray(H, dtype=np.float64)
    return (np.asarray(F, dtype=np.float64) + d * (transition_sparse(g_new) @ H)
            - d * (transition_sparse(g_old) @ H))


def set_step_signed(g, d: float, theta: float, F, H):
    """One set step on fluid of either sign: S = {i : F_i != 0, |F_i| >= theta};
    H += F on S, F = 0 on S, then F += d P (the fluid sent).  Returns
    (F', H', taken mask)."""
    F = np.array(F, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    S = (F != 0.0) & (np.abs(F) >= theta)
    sent = np.where(S, F, 0.0)
    H += sent
    F -= sent
    F += d * (transition_sparse(g) @ sent)
    return F, H, S


# ----------------------------------------------------------- weighted graphs

def transition_dense_weighted(g, w) -> np.ndarray:
    """Dense P for a weighted graph: P[j, i] = sum of the weights w_e of the
    links e = i -> j (each non-empty column sums to one; Section 2.1 allows any
    such P).  Dangling columns are zero."""
    n, rp, ci = _csr(g)
    w = np.asarray(w, dtype=np.float64)
    P = np.zeros((n, n))
    for i in range(n):
        for e in range(rp[i], rp[i + 1]):
            P[ci[e], i] += w[e]
    return P


def dense_exact_weighted(g, w, d: float, v=None):
    """(Y, x*) of dense_exact for the weighted P."""
    n = int(g.n)
    v = _v(n, v)
    Y = np.linalg.solve(np.eye(n) - d * transition_dense_weighted(g, w), (1.0 - d) * v)
    return Y, Y / np.abs(Y).sum()


def set_step_weighted(g, w, d: float, theta: float, F, H):
    """One set step on a weighted graph: S = {i : F_i != 0, |F_i| >= theta},
    H += F on S, F = 0 on S, F += d P (the fluid sent), P from the weights."""
    import scipy.sparse as sp
    n, rp, ci = _csr(g)
    src = np.repeat(np.arange(n), np.diff(rp))
    P = sp.csc_matrix((np.asarray(w, dtype=np.float64), (ci.astype(np.int64), src)), shape=(n, n))
    F = np.array(F, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    S = (F != 0.0) & (np.abs(F) >= theta)
    sent = np.where(S, F, 0.0)
    H += sent
    F -= sent
    F += d * (P @ sent)
    return F, H, S


def apply_set(g, d: float, S, F, H):
    """Diffuse exactly the set S (boolean mask) from (F, H): H += F on S, F = 0
    on S, F += d P (the fluid sent) -- the set form of the Section 2.2
    recurrences, for replaying a recorded sequence of sets."""
    F = np.array(F, dtype=np.float64)
    H = np.array(H, dtype=np.float64)
    S = np.asarray(S, dtype=bool)
    sent = np.where(S, F, 0.0)
    H += sent
    F -= sent
    F += d * (transition_sparse(g) @ sent)
    return F, H
