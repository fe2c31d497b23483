"""Lanczos recursions on the Liouvillian (oracle).

The paper names the two flavours (Sec. 2.5) but defers their steps to other
references, so the steps below are this project's reading, written from
standard numerical linear algebra:

Non-Hermitian (two-sided) Lanczos biorthogonalisation.  Start q_1 = p_1 =
v / n_1 with n_1 = ||v||.  T_ij = (p_i, L q_j) with T_ii = alpha_i,
T_{i+1,i} = beta_{i+1}, T_{i,i+1} = gamma_{i+1}.  Each step applies L to q_i
and L^dag = J L J to p_i:
    alpha_i = (p_i, L q_i)
    qh = L q_i - alpha_i q_i - gamma_i q_{i-1}
    ph = L^dag p_i - conj(alpha_i) p_i - conj(beta_i) p_{i-1}
    s = (ph, qh), beta_{i+1} = sqrt|s|, gamma_{i+1} = s / beta_{i+1}
    q_{i+1} = qh / beta_{i+1},  p_{i+1} = ph / conj(gamma_{i+1}).
So |gamma| = |beta| (Sec. 5.5).

Pseudo-Hermitian Lanczos: JL is Hermitian (positive definite for a stable
ground state), so L is self-adjoint in the metric S = JL and a standard
Hermitian Lanczos in <a, b>_S = a^dag J L b needs one application of L per
step.  Start w = L v, n_1 = sqrt(v^dag J w), q_1 = v/n_1, Lq_1 = w/n_1:
    alpha_i = (L q_i)^dag J (L q_i)                      (real)
    r = L q_i - alpha_i q_i - beta_i q_{i-1}
    Lr = L r                                            (the one apply)
    beta_{i+1} = sqrt(r^dag J Lr),  gamma = beta
    q_{i+1} = r / beta_{i+1},  L q_{i+1} = Lr / beta_{i+1}.

Both record z_i^l = (u^l, q_i) (Sec. 2.5, below Eq. resolvent_Liouvillian_Lanczos_q;
the argument order is taken so that chi = n_1 sum_i z_i eta_i is the
resolvent element (u, (w - L)^{-1} v)).

Coefficient arrays (0-based step j = 0..M-1): alpha[j] = T[j][j],
beta[j] = T[j+1][j], gamma[j] = T[j][j+1]; the last beta/gamma is the
residual norm beyond the M x M matrix.

Breakdown (the paper gives no rule; this is the project's reading).  With
Lam = the largest kinetic energy |k+q+G|^2/2 on the response spheres as the
scale of L and eps = BREAKDOWN_TOL:
    nH:        |s| <= eps Lam^2 ||p_i|| ||q_i||
    pH start:  v^dag J L v <= eps Lam (v, v)
    pH step:   r^dag J L r <= eps Lam (r, r)   or   (r, r) <= eps^2 Lam^2 (q_i, q_i)
The chain then stops; ``steps_done`` counts the steps whose alpha and z were
recorded (the step that broke down included).

Re-projection (the project's reading of how the recursion stays in the space
L acts on).  The Liouvillian is defined on the empty manifold (the P_c, P_c^+
projectors of Sec. 2.4, Eqs. P_minus_q2 and P_plus_q2); every vector of the
recursion lies in it in exact arithmetic.  In floating point, rounding-level
occupied components creep in; they carry no weight in the metric S = JL (its
null space), so dividing by ever smaller beta amplifies them until
r^dag J L r reaches zero and the pseudo-Hermitian chain breaks down after a
few hundred steps.  The residual r (pH) and the pair q_i, p_i (nH) are
therefore projected again before every application -- the identity in exact
arithmetic.  (A projection only every sixth step was tried and still let
some chains of the 24-q path break down.)
"""
from __future__ import annotations

import numpy as np

BREAKDOWN_TOL = 1e-10
REPROJECT_PH = 1    # steps between re-projections (pH)
REPROJECT_NH = 1    # (nH)


def _result(M, nlam):
    return dict(alpha=np.zeros(M, dtype=np.complex128), beta=np.zeros(M),
                gamma=np.zeros(M, dtype=np.complex128),
                z=np.zeros((nlam, M), dtype=np.complex128), n1=0.0, steps_done=0,
                breakdown=False)


def pseudo_hermitian(apply, v, us, nsteps, dot, J, lam, proj=None):
    eps = BREAKDOWN_TOL
    res = _result(nsteps, len(us))
    w = apply(v)
    n1sq = dot(v, J(w)).real
    if not n1sq > eps * lam * dot(v, v).real:
        res["breakdown"] = True
        return res
    n1 = np.sqrt(n1sq)
    res["n1"] = n1
    q = v / n1
    Lq = w / n1
    q_prev = np.zeros_like(v)
    b_prev = 0.0
    for j in range(nsteps):
        for l, u in enumerate(us):
            res["z"][l, j] = dot(u, q)
        a = dot(Lq, J(Lq)).real
        res["alpha"][j] = a
        r = Lq - a * q - b_prev * q_prev
        if proj is not None and j % REPROJECT_PH == 0:
            r = proj(r)
        Lr = apply(r)
        b2 = dot(r, J(Lr)).real
        rr = dot(r, r).real
        res["steps_done"] = j + 1
        if not (b2 > eps * lam * rr and rr > eps * eps * lam * lam * dot(q, q).real):
            res["breakdown"] = j + 1 < nsteps
            break
        b = np.sqrt(b2)
        res["beta"][j] = b
        res["gamma"][j] = b
        q_prev, q, Lq, b_prev = q, r / b, Lr / b, b
    return res


def non_hermitian(apply, apply_dag, v, us, nsteps, dot, lam, proj=None):
    eps = BREAKDOWN_TOL
    res = _result(nsteps, len(us))
    n1 = np.sqrt(dot(v, v).real)
    if n1 == 0.0:
        res["breakdown"] = True
        return res
    res["n1"] = n1
    q = v / n1
    p = q.copy()
    q_prev = np.zeros_like(v)
    p_prev = np.zeros_like(v)
    b_prev, g_prev = 0.0, 0.0
    for j in range(nsteps):
        if proj is not None and j % REPROJECT_NH == 0:
            q, p = proj(q), proj(p)
        for l, u in enumerate(us):
            res["z"][l, j] = dot(u, q)
        Lq = apply(q)
        Ltp = apply_dag(p)
        a = dot(p, Lq)
        res["alpha"][j] = a
        qh = Lq - a * q - g_prev * q_prev
        ph = Ltp - np.conj(a) * p - np.conj(b_prev) * p_prev
        s = dot(ph, qh)
        res["steps_done"] = j + 1
        scale = np.sqrt(dot(p, p).real * dot(q, q).real)
        if not abs(s) > eps * lam * lam * scale:
            res["breakdown"] = j + 1 < nsteps
            break
        b = np.sqrt(abs(s))
        g = s / b
        res["beta"][j] = b
        res["gamma"][j] = g
        q_prev, p_prev = q, p
        q = qh / b
        p = ph / np.conj(g)
        b_prev, g_prev = b, g
    return res


def run(problem, mu, flavour, nsteps, measure=("x", "y", "z"), reproject=True, **kw):
    """One chain for direction mu on an oracle Problem."""
    v = problem.v_vector(mu)
    us = [problem.u_vector(l) for l in measure]
    apply = lambda x: problem.apply(x, **kw)
    lam = operator_scale(problem)
    proj = problem.project_all if reproject else None
    if flavour in ("pH", "pseudo_hermitian"):
        return pseudo_hermitian(apply, v, us, nsteps, problem.dot, problem.J, lam, proj)
    apply_dag = lambda x: problem.apply_dagger(x, **kw)
    return non_hermitian(apply, apply_dag, v, us, nsteps, problem.dot, lam, proj)


def operator_scale(problem):
    """Lam: the largest kinetic energy on the response spheres."""
    return max(float(kd.kin.max()) for kd in problem.k)
