"""Oracle: limited-memory BFGS minimisation of the EI cost.

TEST INFRASTRUCTURE ONLY (FP64 NumPy, shares no code with the HIP path).

The paper minimises eq. 5 with SciPy's L-BFGS(-B) and states no settings. The reading
implemented here (no bounds, since the paper states none):
  * unknowns are the scaled z (see model.ScaledProblem);
  * memory m pairs (s_i, y_i); search direction d = -H g by the two-loop recursion with
    H_0 = gamma I, gamma = s^T y / y^T y of the newest pair; with empty memory d = -g;
  * if g^T d >= 0 the memory is cleared and d = -g;
  * first trial step alpha = 1/||g|| when the memory is empty, else alpha = 1;
  * Armijo backtracking: accept when F(z + alpha d) <= F(z) + c1 alpha g^T d (c1 = 1e-4),
    otherwise halve alpha, at most max_ls trials;
  * when every trial fails: with non-empty memory, clear it and redo the iteration along
    -g; with empty memory, stop with a line-search failure;
  * the pair s = z_new - z, y = g_new - g is stored only if s^T y > 1e-10 ||s|| ||y||
    (oldest pair dropped beyond m);
  * one iteration = one accepted step; the run stops after max_iter iterations, or earlier
    when ||z_new - z|| / ||z|| < tol_rel_step (if tol_rel_step > 0).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

STATUS_OK = 0
STATUS_LINESEARCH = -6
STATUS_NONFINITE = -5


@dataclass
class LBFGSState:
    z: np.ndarray
    f: float
    g: np.ndarray
    S: list = field(default_factory=list)
    Y: list = field(default_factory=list)
    k: int = 0
    evals: int = 1

    def copy(self):
        return LBFGSState(self.z.copy(), self.f, self.g.copy(), [s.copy() for s in self.S],
                          [y.copy() for y in self.Y], self.k, self.evals)


@dataclass
class Trace:
    cost: list = field(default_factory=list)
    alpha: list = field(default_factory=list)
    trials: list = field(default_factory=list)
    status: int = STATUS_OK


def two_loop(g: np.ndarray, S: list, Y: list) -> np.ndarray:
    """H g for the L-BFGS inverse-Hessian approximation built from the stored pairs."""
    q = np.array(g, dtype=np.float64, copy=True)
    if not S:
        return q
    rho = [1.0 / float(np.dot(y.ravel(), s.ravel())) for s, y in zip(S, Y)]
    alpha = [0.0] * len(S)
    for i in range(len(S) - 1, -1, -1):
        alpha[i] = rho[i] * float(np.dot(S[i].ravel(), q.ravel()))
        q -= alpha[i] * Y[i]
    s, y = S[-1], Y[-1]
    gamma = float(np.dot(s.ravel(), y.ravel())) / float(np.dot(y.ravel(), y.ravel()))
    r = gamma * q
    for i in range(len(S)):
        beta = rho[i] * float(np.dot(Y[i].ravel(), r.ravel()))
        r += S[i] * (alpha[i] - beta)
    return r


def dense_bfgs_inverse(S: list, Y: list, n: int) -> np.ndarray:
    """Explicit BFGS inverse-Hessian recursion H <- V^T H V + rho s s^T from H_0 = gamma I
    (textbook form), used to pin the two-loop recursion."""
    s, y = S[-1].ravel(), Y[-1].ravel()
    H = (s @ y) / (y @ y) * np.eye(n)
    for s, y in zip(S, Y):
        s, y = s.ravel(), y.ravel()
        rho = 1.0 / (y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


def minimize(fun, z0: np.ndarray, max_iter: int, m: int = 10, max_ls: int = 20,
             c1: float = 1e-4, tol_rel_step: float = 0.0, state: LBFGSState | None = None,
             trace: Trace | None = None, callback=None):
    """Run until `max_iter` total iterations (state.k counts across resumes).
    Returns (z, state, trace)."""
    trace = Trace() if trace is None else trace
    if state is None:
        f, g = fun(np.array(z0, dtype=np.float64, copy=True))
        state = LBFGSState(z=np.array(z0, dtype=np.float64, copy=True), f=f, g=g)
        if not np.isfinite(f):
            trace.status = STATUS_NONFINITE
            return state.z, state, trace
    st = state
    while st.k < max_iter:
        if st.S:
            d = -two_loop(st.g, st.S, st.Y)
            alpha = 1.0
        else:
            d = -st.g
            alpha = 1.0 / float(np.linalg.norm(st.g))
        gd = float(np.dot(st.g.ravel(), d.ravel()))
        if not gd < 0.0:
            st.S.clear(); st.Y.clear()
            d = -st.g
            alpha = 1.0 / float(np.linalg.norm(st.g))
            gd = float(np.dot(st.g.ravel(), d.ravel()))
        accepted = False
        trials = 0
        for _ in range(max_ls):
            z_t = st.z + alpha * d
            f_t, g_t = fun(z_t)
            st.evals += 1
            trials += 1
            if f_t <= st.f + c1 * alpha * gd:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            if st.S:
                st.S.clear(); st.Y.clear()
                continue
            trace.status = STATUS_LINESEARCH
            break
        if not np.isfinite(f_t):
            trace.status = STATUS_NONFINITE
            break
        s = z_t - st.z
        y = g_t - st.g
        sy = float(np.dot(s.ravel(), y.ravel()))
        if sy > 1e-10 * float(np.linalg.norm(s)) * float(np.linalg.norm(y)):
            st.S.append(s); st.Y.append(y)
            if len(st.S) > m:
                st.S.pop(0); st.Y.pop(0)
        step = float(np.linalg.norm(s))
        znorm = float(np.linalg.norm(st.z))
        st.z, st.f, st.g = z_t, f_t, g_t
        st.k += 1
        trace.cost.append(f_t); trace.alpha.append(alpha); trace.trials.append(trials)
        if callback is not None:
            callback(st)
        if tol_rel_step > 0.0 and znorm > 0.0 and step / znorm < tol_rel_step:
            break
    return st.z, st, trace


def reconstruct(problem, x0: np.ndarray, max_iter: int, m: int = 10, max_ls: int = 20,
                tol_rel_step: float = 0.0):
    """Raw-unit wrapper: x0 [2][N][N] -> x_K, plus the state and trace."""
    z0 = problem.to_z(x0)
    z, st, tr = minimize(problem, z0, max_iter, m=m, max_ls=max_ls, tol_rel_step=tol_rel_step)
    return problem.to_x(z), st, tr
