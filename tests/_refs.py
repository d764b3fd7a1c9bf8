"""Independent dense references used to pin the oracle (test-side only).

None of these call the oracle or share its code.  They restate the *problem*
(not the closed-form iteration) in dense matrices:

  * velocity_dense   F, G, h of the splitting in the proof of Theorem 2
                     (eqn. (9): F p + G q = h) and the dense cost of f(p);
  * p_subproblem     argmin_p f(p) + rho/2 ||F p + G q - h + s||^2 by a dense
                     linear solve (the first ADMM block before decoupling);
  * q_subproblem     argmin_q g(q) + rho/2 ||F p + G q - h + s||^2 by bounded
                     least squares (scipy BVLS);
  * lqr              finite-horizon discrete Riccati recursion (textbook);
  * eq_qp_original   equality-constrained QP of eqn. (1) in the original
                     (x, u) coordinates solved through its KKT system;
  * qp_admm          the general-QP ADMM of eqn. (3) on the sparse QP (2),
                     an independent algorithm with the same optimum;
  * accel_admm_dense Algorithm 1 with the restart acceleration of steps 6-7,
                     run on the dense splitting with the two sub-problems
                     above.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize


def velocity_dense(p):
    """Dense F, G, h, cost P, linear term qv and box of the velocity-form
    problem (proof of Theorem 2) for a Problem `p`.

    p-vector = (du_0..du_{N-1}, xbar_1..xbar_N); q-vector = (v_0..v_{N-1},
    z_1..z_N); constraint rows grouped (theta_k rows, beta_k rows, lambda_k rows).
    """
    n, m, N = p.nx, p.nu, p.N
    nb = n + m
    A, B, e = p.stage_A(), p.stage_B(), p.stage_e()
    Abar = np.zeros((N, nb, nb))
    Bbar = np.zeros((N, nb, m))
    ebar = np.zeros((N, nb))
    for k in range(N):
        Abar[k][:n, :n] = A[k]
        Abar[k][:n, n:] = B[k]
        Abar[k][n:, n:] = np.eye(m)
        Bbar[k][:n] = B[k]
        Bbar[k][n:] = np.eye(m)
        ebar[k][:n] = e[k]
    npv = N * m + N * nb
    nq = 2 * N * nb
    ns = 3 * N * nb
    F = np.zeros((ns, npv))
    G = np.zeros((ns, nq))
    h = np.zeros(ns)
    du = lambda k: slice(k * m, (k + 1) * m)
    xb = lambda k: slice(N * m + (k - 1) * nb, N * m + k * nb)  # xbar_k, k = 1..N
    vv = lambda k: slice(k * nb, (k + 1) * nb)
    zz = lambda k: slice(N * nb + (k - 1) * nb, N * nb + k * nb)  # z_k, k = 1..N
    th = lambda k: slice(k * nb, (k + 1) * nb)
    be = lambda k: slice(N * nb + k * nb, N * nb + (k + 1) * nb)
    la = lambda k: slice(2 * N * nb + k * nb, 2 * N * nb + (k + 1) * nb)
    I = np.eye(nb)
    xbar0 = p.xbar0()
    for k in range(N):
        # xbar_{k+1} - z_{k+1} = 0
        F[th(k), xb(k + 1)] = I
        G[th(k), zz(k + 1)] = -I
        # Bbar_k du_k - v_k = 0
        F[be(k), du(k)] = Bbar[k]
        G[be(k), vv(k)] = -I
        # z_{k+1} - Abar_k xbar_k - v_k - ebar_k = 0
        G[la(k), zz(k + 1)] = I
        G[la(k), vv(k)] = -I
        if k >= 1:
            F[la(k), xb(k)] = -Abar[k]
            h[la(k)] = ebar[k]
        else:
            h[la(k)] = ebar[k] + Abar[0] @ xbar0
    Qbar = np.zeros((nb, nb))
    Qbar[:n, :n] = p.Q
    Qbar[n:, n:] = p.R
    P = np.zeros((npv, npv))
    qv = np.zeros(npv)
    qbar = np.zeros(nb) if p.qbar is None else np.asarray(p.qbar)
    for k in range(1, N + 1):
        P[xb(k), xb(k)] = Qbar
        qv[xb(k)] = qbar
    if getattr(p, "Wdu", None) is not None:
        for k in range(N):
            P[du(k), du(k)] = p.Wdu
    lo = np.concatenate([np.full(N * nb, -np.inf), np.tile(p.lb(), N)])
    hi = np.concatenate([np.full(N * nb, np.inf), np.tile(p.ub(), N)])
    return dict(F=F, G=G, h=h, P=P, qv=qv, lo=lo, hi=hi, Abar=Abar, Bbar=Bbar, ebar=ebar)


def state_to_qs(state):
    """Oracle state (5, N, nb) = (v, z, theta, beta, lambda) -> dense (q, s)."""
    v, z, th, be, la = state
    q = np.concatenate([v.ravel(), z.ravel()])
    s = np.concatenate([th.ravel(), be.ravel(), la.ravel()])
    return q, s


def qs_to_state(q, s, N, nb):
    v = q[: N * nb].reshape(N, nb)
    z = q[N * nb:].reshape(N, nb)
    th = s[: N * nb].reshape(N, nb)
    be = s[N * nb: 2 * N * nb].reshape(N, nb)
    la = s[2 * N * nb:].reshape(N, nb)
    return np.stack([v, z, th, be, la])


def p_subproblem(D, rho, q, s):
    """argmin_p 1/2 p'Pp - qv'p + rho/2 ||F p + G q - h + s||^2 (dense solve)."""
    F, G, h, P, qv = D["F"], D["G"], D["h"], D["P"], D["qv"]
    M = P + rho * F.T @ F
    rhs = qv - rho * F.T @ (G @ q - h + s)
    return np.linalg.solve(M, rhs)


def q_subproblem(D, rho, pvec, s):
    """argmin_q I_box(z) + rho/2 ||F p + G q - h + s||^2 (bounded least squares)."""
    F, G, h = D["F"], D["G"], D["h"]
    target = h - F @ pvec - s
    lo, hi = D["lo"], D["hi"]
    res = scipy.optimize.lsq_linear(G, target, bounds=(lo, hi), method="bvls", tol=1e-15,
                                    lsmr_tol=None, max_iter=10000)
    return res.x


def lqr(A, B, Q, R, x0, N):
    """Finite-horizon LQR for sum_{k<N} 1/2 x_{k+1}'Q x_{k+1} + 1/2 u_k'R u_k,
    x_{k+1} = A x_k + B u_k.  Returns (x_1..x_N, u_0..u_{N-1})."""
    P = Q.copy()
    Ks = [None] * N
    for k in range(N - 1, -1, -1):
        Kk = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
        Ks[k] = Kk
        P = Q + A.T @ P @ (A - B @ Kk)
    xs, us = [], []
    x = x0.copy()
    for k in range(N):
        u = -Ks[k] @ x
        x = A @ x + B @ u
        us.append(u)
        xs.append(x)
    return np.array(xs), np.array(us)


def original_qp(p):
    """Sparse QP (2) of problem (1) in original coordinates y = col(u_0, x_1,
    ..., u_{N-1}, x_N): cost 1/2 y'Hy + f'y, equality rows Aeq y = beq
    (dynamics), box rows on every u and x.  An input-rate weight Wdu adds
    sum_k 1/2 (u_k - u_{k-1})'Wdu(u_k - u_{k-1}) with u_{-1} = u_prev.
    Returns dict."""
    n, m, N = p.nx, p.nu, p.N
    A, B, e = p.stage_A(), p.stage_B(), p.stage_e()
    ny = N * (n + m)
    uu = lambda k: slice(k * (n + m), k * (n + m) + m)
    xx = lambda k: slice(k * (n + m) + m, (k + 1) * (n + m))  # x_{k+1}
    H = np.zeros((ny, ny))
    f = np.zeros(ny)
    for k in range(N):
        H[uu(k), uu(k)] = p.R
        H[xx(k), xx(k)] = p.Q
    Wd = getattr(p, "Wdu", None)
    if Wd is not None:
        for k in range(N):
            H[uu(k), uu(k)] += Wd
            if k >= 1:
                H[uu(k - 1), uu(k - 1)] += Wd
                H[uu(k), uu(k - 1)] -= Wd
                H[uu(k - 1), uu(k)] -= Wd
            else:
                f[uu(0)] -= Wd @ np.asarray(p.u_prev, np.float64)
    Aeq = np.zeros((N * n, ny))
    beq = np.zeros(N * n)
    for k in range(N):
        r = slice(k * n, (k + 1) * n)
        Aeq[r, xx(k)] = np.eye(n)
        Aeq[r, uu(k)] = -B[k]
        if k >= 1:
            Aeq[r, xx(k - 1)] = -A[k]
            beq[r] = e[k]
        else:
            beq[r] = e[k] + A[0] @ p.x0
    lo = np.zeros(ny)
    hi = np.zeros(ny)
    for k in range(N):
        lo[uu(k)], hi[uu(k)] = p.umin, p.umax
        lo[xx(k)], hi[xx(k)] = p.xmin, p.xmax
    return dict(H=H, f=f, Aeq=Aeq, beq=beq, lo=lo, hi=hi, uu=uu, xx=xx)


def eq_qp_original(p):
    """Equality-constrained QP (bounds ignored) via its KKT system."""
    D = original_qp(p)
    H, Aeq, beq = D["H"], D["Aeq"], D["beq"]
    ny, ne = H.shape[0], Aeq.shape[0]
    K = np.block([[H, Aeq.T], [Aeq, np.zeros((ne, ne))]])
    rhs = np.concatenate([-D["f"], beq])
    sol = np.linalg.solve(K, rhs)
    y = sol[:ny]
    N = p.N
    us = np.array([y[D["uu"](k)] for k in range(N)])
    xs = np.array([y[D["xx"](k)] for k in range(N)])
    return xs, us


def qp_admm(p, rho=1.0, iters=60000, tol=1e-12):
    """General-QP ADMM of eqn. (3) on the sparse QP (2): E = [Aeq; I], Y =
    {beq} x box.  Returns (xs, us, y, w, lam, iters_run)."""
    D = original_qp(p)
    H, Aeq, beq, lo, hi = D["H"], D["Aeq"], D["beq"], D["lo"], D["hi"]
    ny = H.shape[0]
    E = np.vstack([Aeq, np.eye(ny)])
    Ylo = np.concatenate([beq, lo])
    Yhi = np.concatenate([beq, hi])
    Minv = np.linalg.inv(H + rho * E.T @ E)
    w = np.zeros(E.shape[0])
    lam = np.zeros(E.shape[0])
    y = np.zeros(ny)
    it = 0
    for it in range(1, iters + 1):
        y = Minv @ (-D["f"] + rho * E.T @ (w - lam))
        Ey = E @ y
        w_new = np.clip(Ey + lam, Ylo, Yhi)
        lam = lam + Ey - w_new
        r_p = np.max(np.abs(Ey - w_new))
        r_d = rho * np.max(np.abs(E.T @ (w_new - w)))
        w = w_new
        if r_p < tol and r_d < tol:
            break
    N = p.N
    us = np.array([y[D["uu"](k)] for k in range(N)])
    xs = np.array([y[D["xx"](k)] for k in range(N)])
    return dict(xs=xs, us=us, y=y, w=w, lam=lam, iters=it, E=E, H=H, f=D["f"], Ylo=Ylo, Yhi=Yhi,
                rho=rho)


def accel_admm_dense(p, K, eta=0.999, variant=None):
    """Algorithm 1 with steps 6-7 (restart acceleration) on the dense
    splitting of the proof of Theorem 2, written from the algorithm's
    statement rather than from the stage closed forms:

      p^{i+1} = argmin f(p) + rho/2 ||F p + G qhat - h + shat||^2   (dense solve)
      q^{i+1} = argmin I_X(z) + rho/2 ||F p^{i+1} + G q - h + shat||^2 (BVLS)
      s^{i+1} = shat + F p^{i+1} + G q^{i+1} - h
      c^{i+1} = rho ||s^{i+1} - shat||^2 + rho ||G (q^{i+1} - qhat)||^2
      if c^{i+1} <= eta c^i:  alpha' = (1 + sqrt(1 + 4 alpha^2)) / 2,
                              hat = new + (alpha - 1) / alpha' (new - previous)
      else (restart):         alpha' = 1, hat = new (the current iterate)
      c^i <- c^{i+1}, with c^0 = 1 and alpha_0 = 1.

    Cold start.  Returns the actual iterates (q, s) after every iteration and
    the per-iteration c and restart flags.  `variant` deliberately misreads
    the steps, so that a test can show it would notice such a misreading:
    "coef_next" takes (alpha' - 1) / alpha' as the coefficient,
    "restart_prev" resets the hats to the previous iterate on a restart (the
    reading of the pseudo-code (11)), "cprev_kept" leaves c^i unchanged on a
    restart."""
    D = velocity_dense(p)
    N, nb = p.N, p.nx + p.nu
    G = D["G"]
    q = np.zeros(2 * N * nb)
    s = np.zeros(3 * N * nb)
    qh, sh = q.copy(), s.copy()
    alpha, c_prev = 1.0, 1.0
    qs, ss, cs, restarts = [], [], [], []
    for _ in range(K):
        pv = p_subproblem(D, p.rho, qh, sh)
        qn = q_subproblem(D, p.rho, pv, sh)
        sn = sh + D["F"] @ pv + G @ qn - D["h"]
        c = p.rho * float(np.sum((sn - sh) ** 2)) + p.rho * float(np.sum((G @ (qn - qh)) ** 2))
        if c <= eta * c_prev:
            a1 = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * alpha * alpha))
            coef = (a1 - 1.0) / a1 if variant == "coef_next" else (alpha - 1.0) / a1
            qh = qn + coef * (qn - q)
            sh = sn + coef * (sn - s)
            alpha = a1
            restarts.append(0)
        else:
            alpha = 1.0
            if variant == "restart_prev":
                qh, sh = q.copy(), s.copy()
            else:
                qh, sh = qn.copy(), sn.copy()
            restarts.append(1)
        if not (variant == "cprev_kept" and restarts[-1]):
            c_prev = c
        q, s = qn, sn
        qs.append(q.copy())
        ss.append(s.copy())
        cs.append(c)
    return dict(q=qs, s=ss, c=np.array(cs), restart=np.array(restarts), eta=eta)


def sparse_qp(p):
    """QP (2) of problem (1) as scipy.sparse matrices, in the same original
    coordinates y = col(u_0, x_1, ..., u_{N-1}, x_N) as `original_qp`, for
    horizons where dense matrices do not fit.  The linear term qbar of the
    velocity-form cost (-qbar' xbar_{k+1}, xbar_{k+1} = col(x_{k+1}, u_k)), an
    input-rate weight Wdu, and the output form of eqn. (1) (outputs w_k =
    C x_{k+1} as extra variables with their weight, reference and bounds; an
    input reference) are included."""
    import scipy.sparse as sp
    n, m, N = p.nx, p.nu, p.N
    nb = n + m
    A, B, e = p.stage_A(), p.stage_B(), p.stage_e()
    ny = N * nb
    Hr, Hc, Hv = [], [], []

    def blk(r0, c0, M):
        M = np.asarray(M, np.float64)
        rr, cc = np.nonzero(M)
        Hr.extend(rr + r0)
        Hc.extend(cc + c0)
        Hv.extend(M[rr, cc])

    f = np.zeros(ny)
    Wd = getattr(p, "Wdu", None)
    qb = None if p.qbar is None else np.asarray(p.qbar, np.float64)
    for k in range(N):
        u0, x0 = k * nb, k * nb + m
        blk(u0, u0, p.R)
        blk(x0, x0, p.Q)
        if qb is not None:
            f[x0:x0 + n] -= qb[:n]
            f[u0:u0 + m] -= qb[n:]
        if Wd is not None:
            blk(u0, u0, Wd)
            if k >= 1:
                blk(u0 - nb, u0 - nb, Wd)
                blk(u0, u0 - nb, -np.asarray(Wd))
                blk(u0 - nb, u0, -np.asarray(Wd))
            else:
                f[u0:u0 + m] -= np.asarray(Wd) @ np.asarray(p.u_prev, np.float64)
    # output form of eqn. (1): extra variables w_k = C x_{k+1} (after the
    # N (n + m) block) carry 1/2 ||w - ry||^2_Wy and the output bounds; the
    # input reference adds 1/2 ||u - ru||^2_R - 1/2 u'R u = -(R ru)'u (+ const)
    C = getattr(p, "C", None)
    nyo = 0 if C is None else int(np.asarray(C).shape[0])
    nw = N * nyo
    if nyo:
        Wy = np.asarray(p.Wy, np.float64)
        ry = np.zeros(nyo) if getattr(p, "ry", None) is None else np.asarray(p.ry, np.float64)
        for k in range(N):
            blk(ny + k * nyo, ny + k * nyo, Wy)
        f = np.concatenate([f, np.tile(-Wy @ ry, N)])
    if getattr(p, "ru", None) is not None:
        fu = -np.asarray(p.R, np.float64) @ np.asarray(p.ru, np.float64)
        for k in range(N):
            f[k * nb:k * nb + m] += fu
    H = sp.csc_matrix((Hv, (Hr, Hc)), shape=(ny + nw, ny + nw))
    Ar, Ac, Av = [], [], []
    beq = np.zeros(N * n + nw)
    for k in range(N):
        r0, u0, x0 = k * n, k * nb, k * nb + m
        for i in range(n):
            Ar.append(r0 + i); Ac.append(x0 + i); Av.append(1.0)
            for j in range(m):
                if B[k][i, j] != 0.0:
                    Ar.append(r0 + i); Ac.append(u0 + j); Av.append(-B[k][i, j])
            if k >= 1:
                for j in range(n):
                    if A[k][i, j] != 0.0:
                        Ar.append(r0 + i); Ac.append(x0 - nb + j); Av.append(-A[k][i, j])
        beq[r0:r0 + n] = e[k] + (A[0] @ p.x0 if k == 0 else 0.0)
    if nyo:
        Cm = np.asarray(C, np.float64)
        for k in range(N):
            for a in range(nyo):
                row = N * n + k * nyo + a
                Ar.append(row); Ac.append(ny + k * nyo + a); Av.append(1.0)
                for j in range(n):
                    if Cm[a, j] != 0.0:
                        Ar.append(row); Ac.append(k * nb + m + j); Av.append(-Cm[a, j])
    Aeq = sp.csc_matrix((Av, (Ar, Ac)), shape=(N * n + nw, ny + nw))
    lo = np.tile(np.concatenate([p.umin, p.xmin]).astype(np.float64), N)
    hi = np.tile(np.concatenate([p.umax, p.xmax]).astype(np.float64), N)
    if nyo:
        ylo = np.full(nyo, -np.inf) if getattr(p, "ymin", None) is None else np.asarray(p.ymin, np.float64)
        yhi = np.full(nyo, np.inf) if getattr(p, "ymax", None) is None else np.asarray(p.ymax, np.float64)
        lo = np.concatenate([lo, np.tile(ylo, N)])
        hi = np.concatenate([hi, np.tile(yhi, N)])
    return dict(H=H, f=f, Aeq=Aeq, beq=beq, lo=lo, hi=hi, nb=nb)


def ipm_qp(p, tol=1e-12, max_iter=80):
    """Optimum of QP (2) by a primal-dual interior-point method (Mehrotra's
    predictor-corrector, textbook form; infeasible start, slacks for every
    finite bound), each Newton system solved by a sparse LU of the
    quasi-definite KKT matrix.  An algorithm unrelated to ADMM, for a KKT
    point of long horizons.  Returns dict(xs (N,n), us (N,m), y, kkt = the
    largest scaled residual, iters, ok)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    D = sparse_qp(p)
    H, f, Aeq, beq, lo, hi = D["H"], D["f"], D["Aeq"], D["beq"], D["lo"], D["hi"]
    ny, ne = H.shape[0], Aeq.shape[0]
    il = np.flatnonzero(np.isfinite(lo))
    iu = np.flatnonzero(np.isfinite(hi))
    y = np.zeros(ny)
    both = np.isfinite(lo) & np.isfinite(hi)
    y[both] = 0.5 * (lo[both] + hi[both])
    sl = np.maximum(y[il] - lo[il], 1.0)
    su = np.maximum(hi[iu] - y[iu], 1.0)
    zl = np.ones(il.size)
    zu = np.ones(iu.size)
    nu_ = np.zeros(ne)
    AT = Aeq.T.tocsc()
    nbound = il.size + iu.size
    ok = False
    it = 0
    kkt = np.inf
    scale = 1.0 + max(np.max(np.abs(f)), np.max(np.abs(beq)))
    for it in range(1, max_iter + 1):
        rd = H @ y + f - AT @ nu_
        rd[il] -= zl
        rd[iu] += zu
        re = Aeq @ y - beq
        rl = y[il] - lo[il] - sl
        ru = hi[iu] - y[iu] - su
        mu = (sl @ zl + su @ zu) / max(nbound, 1)
        kkt = max(np.max(np.abs(rd)), np.max(np.abs(re)), np.max(np.abs(rl), initial=0.0),
                  np.max(np.abs(ru), initial=0.0), mu) / scale
        if kkt <= tol:
            ok = True
            break
        sig = np.zeros(ny)
        np.add.at(sig, il, zl / sl)
        np.add.at(sig, iu, zu / su)
        Kmat = sp.bmat([[H + sp.diags(sig), AT], [Aeq, None]], format="csc")
        lu = spla.splu(Kmat)

        def step(cl, cu):
            # complementarity targets sl zl -> cl, su zu -> cu
            r1 = -rd.copy()
            r1[il] += (cl - zl * rl) / sl - zl + zl * 0.0
            r1[iu] -= (cu - zu * ru) / su - zu
            # r1 built from: -rd + Pl[(cl)/sl - zl - (zl/sl) rl] - Pu[(cu)/su - zu - (zu/su) ru]
            sol = lu.solve(np.concatenate([r1, -re]))
            dy = sol[:ny]
            dsl = dy[il] + rl
            dsu = -dy[iu] + ru
            dzl = (cl - sl * zl - zl * dsl) / sl
            dzu = (cu - su * zu - zu * dsu) / su
            dnu = -sol[ny:]
            return dy, dsl, dsu, dzl, dzu, dnu

        def maxstep(x, dx):
            neg = dx < 0
            return min(1.0, float(np.min(-x[neg] / dx[neg]))) if np.any(neg) else 1.0

        # predictor (affine scaling)
        dy, dsl, dsu, dzl, dzu, dnu = step(np.zeros(il.size), np.zeros(iu.size))
        ap = min(maxstep(sl, dsl), maxstep(su, dsu))
        ad = min(maxstep(zl, dzl), maxstep(zu, dzu))
        mu_aff = ((sl + ap * dsl) @ (zl + ad * dzl) + (su + ap * dsu) @ (zu + ad * dzu)) / max(nbound, 1)
        sigma = (mu_aff / mu) ** 3 if mu > 0 else 0.0
        # corrector with Mehrotra's second-order term
        cl = sigma * mu - dsl * dzl
        cu = sigma * mu - dsu * dzu
        dy, dsl, dsu, dzl, dzu, dnu = step(cl, cu)
        ap = 0.99 * min(maxstep(sl, dsl), maxstep(su, dsu))
        ad = 0.99 * min(maxstep(zl, dzl), maxstep(zu, dzu))
        ap, ad = min(ap, 1.0), min(ad, 1.0)
        y += ap * dy
        sl += ap * dsl
        su += ap * dsu
        zl += ad * dzl
        zu += ad * dzu
        nu_ += ad * dnu
    nb, m = D["nb"], p.nu
    Y = y[:p.N * nb].reshape(p.N, nb)
    return dict(xs=Y[:, m:].copy(), us=Y[:, :m].copy(), y=y, kkt=kkt, iters=it, ok=ok)
