"""Polynomial vector extrapolation (RRE, MPE) and the restarted driver (FP64).

Paper: Section 3, eqs. (8)-(11) (the extrapolated sequence, its Schur-complement
form and the Moore-Penrose form of RRE); Section 3.1, Algorithms 3 (RRE) and 4
(MPE) by QR factorisation of the first differences; Section 3.2, Algorithm 5
(restarted extrapolation).

Readings where the paper is garbled or silent:
  * The restart number q: one restart cycle applies the fixed-point map q+1
    times (s_1 .. s_{q+1} from s_0) and extrapolates from q+1 differences.
  * RRE's eta_{i,j} in eq. (8) is read as (Delta^2 s_i, Delta s_j), so that
    eq. (8), eq. (10) and Algorithm 3 all describe min ||sum gamma_j Delta s_j||
    subject to sum gamma_j = 1.
  * Algorithm 4 solves for d_0 .. d_{q-1} and then sets d_q = 1; gamma_i = d_i/lambda.
  * The inner counter of Algorithm 5 restarts at 0 in every cycle.
  * Breakdown: if |R_jj| <= 1e-13 ||Delta s_j|| for a first column j (Delta s_j
    numerically in the span of the earlier differences), both methods use
    columns 0..j and gamma proportional to (-R_{<j}^{-1} R_{<j, j}, 1), which is
    the exact fixed point of a linear map.  If |lambda| <= 1e-14 ||d||_1 the cycle
    breaks down: no extrapolation, continue from s_{q+1}.
  * Accuracy test: ||b - A t||_2 / ||b||_2 <= tol, applied to t only.
"""
import numpy as np

LUCKY_TOL = 1e-13
LAMBDA_TOL = 1e-14

RRE = "rre"
MPE = "mpe"


class Breakdown(Exception):
    pass


def differences(S):
    """Delta S_{q+1} = [s_1 - s_0, ..., s_{q+1} - s_q] as an N x (q+1) array."""
    S = [np.asarray(s, dtype=np.float64) for s in S]
    return np.column_stack([S[i + 1] - S[i] for i in range(len(S) - 1)])


def _gamma_from_R(R, method):
    """Weights gamma (summing to 1) from the triangular factor R of the
    difference matrix U = Delta S = Q R (so U^T U = R^T R).

    RRE: gamma minimises ||U gamma|| over sum(gamma) = 1.  Stationarity of
    ||U gamma||^2 - 2 lam (sum(gamma) - 1) gives U^T U gamma = lam 1, so gamma
    is d = (R^T R)^{-1} 1 scaled to sum 1.
    MPE: the combination U c with c_q = 1 is orthogonal to the first q
    differences, U_q^T U c = 0, i.e. (R_q^T R_q) c_{<q} = -R_q^T r_q with R_q the
    leading q x q block and r_q the first q entries of the last column; with
    R_q invertible that is R_q c_{<q} = -r_q; gamma = c scaled to sum 1.
    Returns (gamma, info) with info in {"ok", "lucky"}.
    """
    q1 = R.shape[1]
    colnorm = np.sqrt(np.sum(R * R, axis=0))
    for j in range(q1):
        if abs(R[j, j]) <= LUCKY_TOL * colnorm[j]:
            # lucky breakdown: the first j+1 differences are dependent, and the
            # combination of them that vanishes gives the fixed point of a
            # linear map exactly
            if j == 0:
                g = np.zeros(q1)
                g[0] = 1.0
                return g, "lucky"
            d = np.zeros(q1)
            d[:j] = np.linalg.solve(np.triu(R[:j, :j]), -R[:j, j])
            d[j] = 1.0
            lam = d.sum()
            if abs(lam) <= LAMBDA_TOL * np.abs(d).sum():
                raise Breakdown("lambda ~ 0")
            return d / lam, "lucky"
    if method == RRE:
        # (R^T R) d = 1 through the two triangular factors (not the normal
        # matrix, whose condition is the square of R's)
        d = np.linalg.solve(np.triu(R), np.linalg.solve(np.triu(R).T, np.ones(q1)))
    elif method == MPE:
        q = q1 - 1
        d = np.zeros(q1)
        if q > 0:
            d[:q] = np.linalg.solve(np.triu(R[:q, :q]), -R[:q, q])
        d[q] = 1.0
    else:
        raise ValueError(method)
    lam = d.sum()
    if not np.isfinite(lam) or abs(lam) <= LAMBDA_TOL * np.abs(d).sum():
        raise Breakdown("lambda ~ 0")
    return d / lam, "ok"


def _factor(S):
    """Q, R of the difference matrix (Householder QR through numpy), padded to
    q+1 columns when there are fewer unknowns than differences (the missing
    rows of R are zero: the trailing differences are dependent)."""
    U = differences(S)
    q1 = U.shape[1]
    Q, R = np.linalg.qr(U, mode="reduced")
    if R.shape[0] < q1:
        R = np.vstack([R, np.zeros((q1 - R.shape[0], q1))])
        Q = np.hstack([Q, np.zeros((Q.shape[0], q1 - Q.shape[1]))])
    if not np.all(np.isfinite(R)):
        raise FloatingPointError("non-finite R")
    return Q, R


def extrapolate(S, method):
    """The extrapolated vector of s_0 .. s_{q+1} (Section 3, Algorithms 3 and 4):
    t = sum_{j=0}^{q} gamma_j s_j with the RRE or MPE weights of the q+1 first
    differences (see _gamma_from_R).  Returns (t, gamma, info)."""
    _, R = _factor(S)
    gamma, info = _gamma_from_R(R, method)
    t = np.zeros_like(np.asarray(S[0], dtype=np.float64))
    for j in range(len(gamma)):
        t = t + gamma[j] * np.asarray(S[j], dtype=np.float64)
    return t, gamma, info


def extrapolate_qr_form(S, method):
    """The same t computed through the QR factor, as the algorithms do and as
    the library does without forming Q: t = s_0 + sum_{j<q} a_j (s_{j+1} - s_j)
    with a_j = 1 - (gamma_0 + ... + gamma_j), here evaluated as s_0 + Q_q (R_q a)
    (Q_q R_q = U_q, the first q differences).  Equal to extrapolate() up to
    rounding (summation by parts); a cross-check of that identity."""
    Q, R = _factor(S)
    gamma, info = _gamma_from_R(R, method)
    q = len(gamma) - 1
    a = 1.0 - np.cumsum(gamma[:q])
    t = np.asarray(S[0], dtype=np.float64) + Q[:, :q] @ (R[:q, :q] @ a)
    return t, gamma, info


def generalized_residual(S, gamma):
    """Generalised residual of t (Section 3, eq. (11)): r~(t) = t~ - t with
    t = sum_j gamma_j s_j and t~ = sum_j gamma_j s_{j+1}, i.e. sum_j gamma_j Delta s_j."""
    S = [np.asarray(x, dtype=np.float64) for x in S]
    q1 = len(gamma)
    t = sum(gamma[j] * S[j] for j in range(q1))
    tt = sum(gamma[j] * S[j + 1] for j in range(q1))
    return tt - t


def generalized_residual_closed(S, method):
    """The closed form of eq. (11): Delta s_0 - Delta^2 S (Y^T Delta^2 S)^{-1} Y^T Delta s_0
    with Y = Delta^2 S (RRE) or Delta S (MPE), q columns each."""
    U = differences(S)
    d2S = U[:, 1:] - U[:, :-1]
    Y = d2S if method == RRE else U[:, :-1]
    return U[:, 0] - d2S @ np.linalg.solve(Y.T @ d2S, Y.T @ U[:, 0])


def extrapolate_schur(S, method):
    """Closed form eq. (9): t = s_0 - Delta S (Y^T Delta^2 S)^{-1} Y^T Delta s_0.

    Uses Delta S_{0,q}, Delta^2 S_{0,q} (q columns each) and Y = Delta^2 S for
    RRE, Y = Delta S for MPE.  For cross-checking Algorithms 3 and 4.
    """
    U = differences(S)          # q+1 columns: Delta s_0 .. Delta s_q
    dS = U[:, :-1]              # Delta S_{0,q}
    d2S = U[:, 1:] - U[:, :-1]  # Delta^2 S_{0,q}
    Y = d2S if method == RRE else dS
    coef = np.linalg.solve(Y.T @ d2S, Y.T @ U[:, 0])
    return np.asarray(S[0], dtype=np.float64) - dS @ coef


def extrapolate_pinv(S):
    """RRE by the Moore-Penrose form eq. (10): t = s_0 - Delta S (Delta^2 S)^+ Delta s_0."""
    U = differences(S)
    dS = U[:, :-1]
    d2S = U[:, 1:] - U[:, :-1]
    return np.asarray(S[0], dtype=np.float64) - dS @ (np.linalg.pinv(d2S) @ U[:, 0])


class SolveStats:
    def __init__(self):
        self.restarts = 0
        self.vcycles = 0
        self.breakdowns = 0
        self.rel_residual = np.inf
        self.history = []
        self.converged = False


def restarted_solve(G, residual_norm, s0, q, method, tol=1e-10, max_restarts=100,
                    keep_iterates=False):
    """Restarted extrapolation (Section 3.2, Algorithm 5): from the current
    vector, apply the fixed-point map G q+1 times, extrapolate, test the
    extrapolated vector's relative residual and, if it is not small enough,
    start the next cycle from it.  A cycle whose weights are undefined
    (Breakdown) continues from its last iterate.

    G(x) returns the next iterate; residual_norm(x) returns ||b - A x|| / ||b||.
    method None gives the plain iteration, tested after every application of G.
    Returns (x, stats, iterates) where iterates lists every s_j and t produced
    (when keep_iterates).
    """
    st = SolveStats()
    its = []
    x = np.array(s0, dtype=np.float64, copy=True)
    if method is None:
        for k in range(max_restarts):
            x = G(x)
            st.vcycles += 1
            if keep_iterates:
                its.append(x.copy())
            rel = residual_norm(x)
            st.history.append(rel)
            st.rel_residual = rel
            if rel <= tol:
                st.converged = True
                break
        st.restarts = st.vcycles
        return x, st, its
    for k in range(max_restarts):
        S = [x]
        for i in range(q + 1):
            S.append(G(S[-1]))
            st.vcycles += 1
        if keep_iterates:
            its.extend(s.copy() for s in S[1:])
        try:
            t, _, _ = extrapolate(S, method)
        except Breakdown:
            st.breakdowns += 1
            t = S[-1]
        if keep_iterates:
            its.append(t.copy())
        st.restarts += 1
        rel = residual_norm(t)
        st.history.append(rel)
        st.rel_residual = rel
        x = t
        if rel <= tol:
            st.converged = True
            break
    return x, st, its
