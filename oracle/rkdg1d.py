"""The paper's own 1D discretisation, as a plain FP64 NumPy/SciPy reference:
second-order Runge-Kutta discontinuous Galerkin with P1 elements for the
hydrostatic predictor (Sec. 3.1, the weak form Eq. 6, its semi-discrete form
Eq. 7, Heun as Eqs. 8-9) and the local discontinuous Galerkin (LDG) P1
solution of the first-order elliptic system of Eqs. 14-15 with the flip-flop
flux of Eqs. 16-17 (Sec. 3.2), then the correction of Eqs. 10-11.

TEST INFRASTRUCTURE ONLY: imported by tests/.  It shares no code with the
HIP library (nor with oracle/swe_oracle.c beyond the body's motion law, which
the C oracle's pinned routine supplies).

Readings where the paper is silent or garbled (each one is listed in the
design notes):
  * P1 nodal Lagrange basis on each element [x_i, x_{i+1}] with its nodes at
    the element's ends; consistent mass matrix M = dx/6 [[2, 1], [1, 2]] and
    D_jk = int phi_j (phi_k)_x = [[-1/2, 1/2], [-1/2, 1/2]].
  * The semi-discrete form with the source on the right-hand side (the
    printed Eq. 7 places it with the wrong sign): M dQ/dt = int phi_x F(Q_h)
    - [phi F*] + int phi S(Q_h).  No slope limiter (the paper names none).
  * The element integrals of the flux F(Q_h) and of the source
    S = (0, g h d_x, 0) by three-point Gauss-Legendre quadrature of the P1
    state, with d_x the slope of the bottom's P1 interpolant.  Interpolating
    F and S at the nodes instead (the other reading of "approximated
    similarly") is not well balanced: over a fixed quartic block of the
    flume of Sec. 4.3 it moves still water by 1.2e-2 m in 1.5 s at
    dx = 0.075 m, three times the wave the moving block makes.  With
    quadrature, still water stays still (the integrals of g h h_x and of
    (g h^2 / 2)_x agree exactly for a P1 depth).  The products of the
    elliptic system are interpolated at the nodes.
  * Rusanov interface flux; reflective walls (mirror states: hu changes sign).
  * Heun as printed: stage 2 with the bottom at t^{n+1}.
  * LDG flux constants: 1/2 on the own-variable jumps ([p] in p*, [hu] in
    (hu)*; Eqs. 16-17 write [u_h], read as [(hu)_h]) and 0 on the cross
    terms, so p* = p+ (the right element's value) and (hu)* = (hu)- (the
    left element's).  Zero Dirichlet p at both walls (p* = 0 there) with
    (hu)* the interior value; at the left wall, where the alternating flux
    would take p from inside, (hu)* carries the LDG penalty of the Dirichlet
    datum in the form of Eq. 16, (hu)* = (hu)+ + c11 [p] with [p] = 0 - p+
    and c11 = 1 / (s12 dx) > 0 (Castillo, Cockburn, Perugia and Schoetzau
    2000, in the units of hu).  Without it the first element's p oscillates
    about its mean and p converges at first order only; with it both fields
    converge at second order (the opposite sign makes the coupled steps
    unstable at the wall).
  * The bottom d = d_s - B(x - X(t)) with a flat static depth d_s; d and its
    derivatives at the nodes from the body's shape (Eq. 20 quartic, or a
    Gaussian) and its motion law by the chain rule.
  * hw corrected with Eq. 11 after eliminating (h p)_x through Eq. 10:
    P_b = 3 p / 2 - rho d_x (hu - hu~) / (4 dt) + (4 + d_x^2) phi / 4, node by
    node.
  * The adaptive model (Sec. 5) on elements: an element is non-hydrostatic
    when the criterion exceeds k_nh at one of its two nodes (strictly), the
    derivative criteria taking the element's P1 slope; the set is widened by
    e elements on each side (Sec. 5.2); |w| and |w_x| may treat the first
    step as global (Sec. 5.1.2, for initial data at rest; off for the
    solitary wave, whose initial w is not zero).  The LDG system is the global one's rows of the
    marked elements' node unknowns with the others fixed at the zero
    non-hydrostatic state, p = 0 and hu = hu~ (the zero Dirichlet condition
    of Sec. 5.2): across a face into an unmarked element the alternating
    flux takes p from the right (0 at a segment's right end) and hu from the
    left (hu~ at its left end).  Unmarked elements keep the predictor's
    state.  Every element marked is the global model exactly.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import body_motion

G, RHO = 9.81, 1000.0
# P1 element matrices on the reference element of width 1 (scale M by dx)
M_REF = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
D_MAT = np.array([[-0.5, 0.5], [-0.5, 0.5]])  # D_jk = int phi_j (phi_k)_x


def node_x(n, dx):
    """node coordinates [n, 2]: element i spans [i dx, (i + 1) dx]"""
    x0 = np.arange(n) * dx
    return np.stack([x0, x0 + dx], axis=1)


def body_shape(body, xi):
    """B, B', B'' of the body's profile at offsets xi from its centre"""
    xi = np.asarray(xi, dtype=np.float64)
    z = np.zeros_like(xi)
    if body.kind == 1:  # quartic slide, Eq. 20: H (1 - (2 xi / L)^4) on |xi| < L / 2
        L, H = body.length, body.amp
        s = 2.0 * xi / L
        inside = np.abs(xi) < 0.5 * L
        B = np.where(inside, H * (1.0 - s ** 4), z)
        B1 = np.where(inside, -H * 4.0 * s ** 3 * (2.0 / L), z)
        B2 = np.where(inside, -H * 12.0 * s ** 2 * (2.0 / L) ** 2, z)
        return B, B1, B2
    if body.kind == 2:  # Gaussian mound A exp(-xi^2 / w^2)
        w2 = body.length ** 2
        e = body.amp * np.exp(-xi * xi / w2)
        return e, -2.0 * xi / w2 * e, (4.0 * xi * xi / (w2 * w2) - 2.0 / w2) * e
    return z, z, z


def bottom(d_static, body, x, t):
    """d, d_x, d_xx, d_t, d_tt, d_xt at the points x (flat static depth)"""
    X, Xd, Xdd = body_motion(body, t) if body.kind else (0.0, 0.0, 0.0)
    B, B1, B2 = body_shape(body, x - X)
    return (d_static - B, -B1, -B2, Xd * B1, Xdd * B1 - Xd * Xd * B2, Xd * B2)


def _flux(h, m, k, g):
    return np.stack([m, m * m / h + 0.5 * g * h * h, m * k / h])


def _rusanov(qm, qp, g):
    """Rusanov flux between the states qm (left) and qp (right), each [3, nf]"""
    fm, fp = _flux(*qm, g), _flux(*qp, g)
    lam = np.maximum(np.abs(qm[1] / qm[0]) + np.sqrt(g * qm[0]),
                     np.abs(qp[1] / qp[0]) + np.sqrt(g * qp[0]))
    return 0.5 * (fm + fp) - 0.5 * lam * (qp - qm)


# three-point Gauss-Legendre rule on [0, 1]
GAUSS_X = np.array([0.5 - 0.5 * math.sqrt(0.6), 0.5, 0.5 + 0.5 * math.sqrt(0.6)])
GAUSS_W = np.array([5.0, 8.0, 5.0]) / 18.0
PHI_G = np.stack([1.0 - GAUSS_X, GAUSS_X], axis=1)     # phi_j at the points [3, 2]


def operator(Q, dx, slope, g=G):
    """H(Q) of the semi-discrete form: dQ/dt at the nodes.  Q: [3, n, 2]
    (h, hu, hw at each element's two nodes); slope: [n] d_x of the bottom's
    P1 interpolant on each element"""
    if np.any(Q[0] <= 0.0):
        raise FloatingPointError("dry node")
    Qg = np.einsum("gk,ank->ang", PHI_G, Q)               # state at the Gauss points
    Fg = _flux(Qg[0], Qg[1], Qg[2], g)                    # [3, n, 3]
    mirror = np.array([1.0, -1.0, 1.0])[:, None]
    qm = np.concatenate([Q[:, :1, 0] * mirror, Q[:, :, 1]], axis=1)   # left states of faces 0..n
    qp = np.concatenate([Q[:, :, 0], Q[:, -1:, 1] * mirror], axis=1)  # right states
    Fs = _rusanov(qm, qp, g)                             # [3, n + 1]
    # int (phi_j)_x F dx = (+-1) sum_g w_g F_g  ((phi_0)_x = -1/dx, (phi_1)_x = 1/dx)
    fint = np.einsum("g,ang->an", GAUSS_W, Fg)
    rhs = np.stack([-fint, fint], axis=2)
    rhs[:, :, 0] += Fs[:, :-1]                           # -phi_0(x_l) (-F*_l)
    rhs[:, :, 1] -= Fs[:, 1:]                            # -phi_1(x_r) F*_r
    # + int phi_j g h d_x dx
    rhs[1] += dx * np.einsum("g,gj,ng->nj", GAUSS_W, PHI_G, g * Qg[0] * slope[:, None])
    Minv = np.linalg.inv(M_REF * dx)
    return np.einsum("jk,ank->anj", Minv, rhs)


def p1_slope(d_nodes, dx):
    return (d_nodes[:, 1] - d_nodes[:, 0]) / dx


def predict(Q, d_static, body, t, dt, dx, g=G):
    """Heun step of the hydrostatic system: Q~ from Q^n over [t, t + dt]"""
    x = node_x(Q.shape[1], dx)
    s0 = p1_slope(bottom(d_static, body, x, t)[0], dx)
    s1 = p1_slope(bottom(d_static, body, x, t + dt)[0], dx)
    H0 = operator(Q, dx, s0, g)
    Qs = Q + dt * H0
    return Q + 0.5 * dt * (H0 + operator(Qs, dx, s1, g))


def ldg_matrix(s11, s12, s21, s22, dx):
    """LDG-P1 matrix of  p_x + s11 p + s12 q = f1,  q_x + s21 q + s22 p = f2
    with p* = p+, q* = q-, p* = 0 and q* interior at the walls.  Unknowns
    [p (2n), q (2n)], node (i, j) at index 2 i + j; coefficients [n, 2]."""
    n = s11.shape[0]
    N2 = 2 * n
    rows, cols, vals = [], [], []

    def add(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    Mloc = M_REF * dx
    for i in range(n):
        for j in range(2):
            rp, rq = 2 * i + j, N2 + 2 * i + j
            for k in range(2):
                # - int (phi_j)_x v = -(D^T v)_j = -D_kj v_k
                add(rp, 2 * i + k, -D_MAT[k, j])
                add(rq, N2 + 2 * i + k, -D_MAT[k, j])
                # + int phi_j (s v)  (products interpolated at the nodes)
                add(rp, 2 * i + k, Mloc[j, k] * s11[i, k])
                add(rp, N2 + 2 * i + k, Mloc[j, k] * s12[i, k])
                add(rq, N2 + 2 * i + k, Mloc[j, k] * s21[i, k])
                add(rq, 2 * i + k, Mloc[j, k] * s22[i, k])
            if j == 1:  # + phi_1(x_r) v*(x_r)
                if i + 1 < n:
                    add(rp, 2 * (i + 1), 1.0)        # p*_r = p+ (next element's first node)
                add(rq, N2 + 2 * i + 1, 1.0)         # q*_r = q- (own last node; wall: interior)
            else:       # - phi_0(x_l) v*(x_l)
                if i > 0:
                    add(rp, 2 * i, -1.0)             # p*_l = p+ (own first node)
                    add(rq, N2 + 2 * (i - 1) + 1, -1.0)  # q*_l = q- (previous element's last node)
                else:                                # wall: p* = 0, q* = q+ - c11 p+
                    add(rq, N2, -1.0)
                    add(rq, 0, 1.0 / (s12[0, 0] * dx))
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * N2, 2 * N2))


def ldg_rhs(f1, f2, dx):
    Mloc = M_REF * dx
    return np.concatenate([(f1 @ Mloc.T).ravel(), (f2 @ Mloc.T).ravel()])


def ldg_solve(s11, s12, s21, s22, f1, f2, dx):
    """(p, q) node values [n, 2] of the LDG-P1 solution"""
    A = ldg_matrix(s11, s12, s21, s22, dx)
    z = spla.spsolve(A.tocsc(), ldg_rhs(f1, f2, dx))
    n = s11.shape[0]
    return z[:2 * n].reshape(n, 2), z[2 * n:].reshape(n, 2)


def nh_coefficients(Qt, d_static, body, t1, dt, dx, g=G, rho=RHO):
    """node values of s11, s12, s21, s22, f1, f2 (Eqs. 12-15) and of d_x,
    alpha, phi at t^{n+1} from the predictor state Qt"""
    n = Qt.shape[1]
    x = node_x(n, dx)
    d, d_x, d_xx, d_t, d_tt, d_xt = bottom(d_static, body, x, t1)
    h, m, k = Qt
    # element-wise P1 derivatives of h~ and eta~ (constant on each element)
    hx = np.repeat(((h[:, 1] - h[:, 0]) / dx)[:, None], 2, axis=1)
    eta = h - d
    ex = np.repeat(((eta[:, 1] - eta[:, 0]) / dx)[:, None], 2, axis=1)
    u = m / h
    al = 4.0 + d_x * d_x
    phi = rho * h / al * (g * d_x * ex - d_tt - 2.0 * u * d_xt - u * u * d_xx)
    s11 = (2.0 * hx - 3.0 * d_x) / (2.0 * h)
    s12 = rho * al / (4.0 * dt * h)
    f1 = al / (4.0 * h) * (phi * d_x + rho / dt * m)
    s21 = -s11
    s22 = 3.0 * dt / (rho * h)
    f2 = -2.0 * d_t - 2.0 * k / h - d_x * m / (2.0 * h) - dt * al * phi / (2.0 * rho * h)
    return dict(s11=s11, s12=s12, s21=s21, s22=s22, f1=f1, f2=f2, d_x=d_x, al=al, phi=phi)


def step(Q, d_static, body, t, dt, dx, g=G, rho=RHO):
    """one step of the global model: predictor, LDG solve, correction.
    Returns (Q^{n+1}, p) with node arrays [3, n, 2] and [n, 2]"""
    Qt = predict(Q, d_static, body, t, dt, dx, g)
    c = nh_coefficients(Qt, d_static, body, t + dt, dt, dx, g, rho)
    p, q = ldg_solve(c["s11"], c["s12"], c["s21"], c["s22"], c["f1"], c["f2"], dx)
    Pb = 1.5 * p - rho * c["d_x"] * (q - Qt[1]) / (4.0 * dt) + c["al"] * c["phi"] / 4.0
    Qn = np.stack([Qt[0], q, Qt[2] + dt / rho * Pb])
    return Qn, p


def solitary_initial(n, dx, a, d, x0, g=G):
    """node values [3, n, 2] of the Serre solitary wave (Sec. 4.1) at t = 0;
    hw from the divergence constraint (Eq. 4) over the flat static bottom"""
    x = node_x(n, dx)
    c = math.sqrt(g * (d + a))
    K = math.sqrt(3.0 * a / (4.0 * d * d * (d + a)))
    xi = K * (x - x0)
    eta = a / np.cosh(xi) ** 2
    eta_x = -2.0 * K * np.tanh(xi) * eta
    h = d + eta
    return np.stack([h, c * eta, -0.5 * c * d * eta_x])


def run(Q, d_static, body, t0, dt, nsteps, dx, g=G, rho=RHO):
    t = t0
    p = np.zeros(Q.shape[1:])
    for _ in range(nsteps):
        Q, p = step(Q, d_static, body, t, dt, dx, g, rho)
        t += dt
    return Q, p, t


# criteria of Sec. 5.1 (the same numbering as the finite-volume oracle)
CRIT_ETA_D, CRIT_ETA_X, CRIT_U, CRIT_U_X, CRIT_W, CRIT_W_X, CRIT_GLOBAL, CRIT_NONE = range(8)


def element_indicator(Qt, d_static, body, t1, dx, crit):
    """per element the criterion of Sec. 5.1 on the predictor state: the
    larger of its two node values (|eta/d|, |u|, |w|), or the magnitude of
    the element's P1 slope (|eta_x|, |u_x|, |w_x|)"""
    n = Qt.shape[1]
    d = bottom(d_static, body, node_x(n, dx), t1)[0]
    h, m, k = Qt
    if crit == CRIT_ETA_D:
        return np.abs((h - d) / d).max(axis=1)
    if crit == CRIT_U:
        return np.abs(m / h).max(axis=1)
    if crit == CRIT_W:
        return np.abs(k / h).max(axis=1)
    f = {CRIT_ETA_X: h - d, CRIT_U_X: m / h, CRIT_W_X: k / h}[crit]
    return np.abs((f[:, 1] - f[:, 0]) / dx)


def element_mask(Qt, d_static, body, t1, dx, crit, k_nh, enlarge, first_step, first_global=True):
    """non-hydrostatic elements (bool [n]): criterion > k_nh, widened by
    enlarge elements on each side"""
    n = Qt.shape[1]
    if crit == CRIT_GLOBAL or (crit in (CRIT_W, CRIT_W_X) and first_step and first_global):
        return np.ones(n, dtype=bool)
    if crit == CRIT_NONE:
        return np.zeros(n, dtype=bool)
    raw = element_indicator(Qt, d_static, body, t1, dx, crit) > k_nh
    out = raw.copy()
    for e in range(1, enlarge + 1):
        out[e:] |= raw[:-e]
        out[:-e] |= raw[e:]
    return out


def ldg_solve_masked(c, q_tilde, mask, dx):
    """(p, q) node values [n, 2]: the LDG system on the marked elements with
    p = 0 and q = q_tilde on the others"""
    n = mask.shape[0]
    A = ldg_matrix(c["s11"], c["s12"], c["s21"], c["s22"], dx).tocsr()
    b = ldg_rhs(c["f1"], c["f2"], dx)
    node = np.repeat(mask, 2)
    inner = np.concatenate([node, node])
    z = np.concatenate([np.zeros(2 * n), q_tilde.ravel()])
    if inner.any():
        I = np.flatnonzero(inner)
        E = np.flatnonzero(~inner)
        rhs = b[I] - A[I][:, E] @ z[E]
        z[I] = spla.spsolve(A[I][:, I].tocsc(), rhs)
    return z[:2 * n].reshape(n, 2), z[2 * n:].reshape(n, 2)


def step_adaptive(Q, d_static, body, t, dt, dx, crit, k_nh=1e-3, enlarge=0, first_step=False,
                  first_global=True, g=G, rho=RHO):
    """one step of the adaptive model: predictor, element mask, LDG solve on
    the marked elements, correction there.  Returns (Q^{n+1}, p, mask)"""
    Qt = predict(Q, d_static, body, t, dt, dx, g)
    mask = element_mask(Qt, d_static, body, t + dt, dx, crit, k_nh, enlarge, first_step,
                        first_global)
    if not mask.any():
        return Qt, np.zeros(Qt.shape[1:]), mask
    c = nh_coefficients(Qt, d_static, body, t + dt, dt, dx, g, rho)
    p, q = ldg_solve_masked(c, Qt[1], mask, dx)
    Pb = 1.5 * p - rho * c["d_x"] * (q - Qt[1]) / (4.0 * dt) + c["al"] * c["phi"] / 4.0
    Qn = np.stack([Qt[0], q, Qt[2] + dt / rho * Pb])
    Qn[:, ~mask] = Qt[:, ~mask]
    return Qn, p, mask


def run_adaptive(Q, d_static, body, t0, dt, nsteps, dx, crit, k_nh=1e-3, enlarge=0,
                 first_global=True, g=G, rho=RHO):
    """nsteps adaptive steps; returns (Q, p, t, marked elements per step)"""
    t = t0
    p = np.zeros(Q.shape[1:])
    counts = []
    for s in range(nsteps):
        Q, p, mask = step_adaptive(Q, d_static, body, t, dt, dx, crit, k_nh, enlarge, s == 0,
                                   first_global, g, rho)
        counts.append(int(mask.sum()))
        t += dt
    return Q, p, t, counts

