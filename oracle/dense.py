"""The paper's matrix form of the linearized OSB-PD operator, assembled densely.

TEST INFRASTRUCTURE ONLY (tiny grids).  This is a second, independent route
to the internal force: instead of the bond loops of ``pd_oracle.c`` it builds
the global matrices of the matrix-based scheme from their per-bond blocks and
multiplies them,

    E      = C_e U                 (Eqs. 2.4, 2.7)
    Theta  = C_theta E             (Eqs. 2.6, 2.10)
    F_int  = K_theta Theta + K_e E (Eqs. 2.5, 2.8, 2.9)
    F_int  = (K^v + K^d) U,  K^v = K_theta C_theta C_e,  K^d = K_e C_e   (Eq. 2.14)

with its own brute-force horizon search.  F_int here is the restoring force
(the peridynamic force of the solver listing), so the positive semi-definite
stiffness is -(K^v + K^d).
"""

from __future__ import annotations

import numpy as np

from .oracle import constants


def bonds_bruteforce(w):
    """Unique bonds (i < j) with 0 < |xi| <= delta inside one specimen."""
    lat = np.zeros((w.n, 3), dtype=np.int64)
    lat[:, : w.dim] = w.lat
    d = lat[None, :, :] - lat[:, None, :]
    xi = d.astype(np.float64) * w.dx
    r = np.sqrt((xi * xi).sum(-1))
    same = w.specimen[:, None] == w.specimen[None, :]
    ok = (r <= w.delta) & (r > 0) & same
    bi, bj = np.nonzero(np.triu(ok, 1))
    return bi, bj, xi[bi, bj], r[bi, bj]


def matrices(w, rho_bond=None, bonds=None):
    """Global C_e (Nb x 3N), C_theta (N x Nb), K_theta (3N x N), K_e (3N x Nb).

    rho_bond: bond status per unique bond (None = all intact); a broken bond
    contributes to none of the four matrices.
    """
    if bonds is None:
        bi, bj, xi, x = bonds_bruteforce(w)
    else:
        bi, bj = bonds
        lat = np.zeros((w.n, 3), dtype=np.int64)
        lat[:, : w.dim] = w.lat
        xi = (lat[bj] - lat[bi]).astype(np.float64) * w.dx
        x = np.sqrt((xi * xi).sum(-1))
    n, nb = w.n, len(bi)
    M = xi / x[:, None]
    V = np.asarray(w.vol, dtype=np.float64)
    # weighted volume, Eq. 1.9 (w = 1), full geometric family
    m = np.zeros(n)
    np.add.at(m, bi, x * x * V[bj])
    np.add.at(m, bj, x * x * V[bi])
    rho = np.ones(nb) if rho_bond is None else np.asarray(rho_bond, dtype=np.float64)
    CE = np.zeros((nb, 3 * n))
    CTH = np.zeros((n, nb))
    KTH = np.zeros((3 * n, n))
    KE = np.zeros((3 * n, nb))
    for b in range(nb):
        if rho[b] == 0:
            continue
        i, j = bi[b], bj[b]
        mat = w.materials[w.specimen[i]]
        k = constants(w.mode_id(), mat.E, mat.nu)
        A, Kc, G = k["A"], k["K"], k["G"]
        Mb = M[b]
        # Eq. 2.7
        CE[b, 3 * i:3 * i + 3] = -Mb
        CE[b, 3 * j:3 * j + 3] = Mb
        # Eq. 2.10
        CTH[i, b] = A * x[b] * V[j] / m[i]
        CTH[j, b] = A * x[b] * V[i] / m[j]
        # Eq. 2.8
        c = (Kc - G / 3.0) * x[b] * V[i] * V[j]
        KTH[3 * i:3 * i + 3, i] += c * Mb / m[i]
        KTH[3 * j:3 * j + 3, i] += -c * Mb / m[i]
        KTH[3 * i:3 * i + 3, j] += c * Mb / m[j]
        KTH[3 * j:3 * j + 3, j] += -c * Mb / m[j]
        # Eq. 2.9
        g = G * V[i] * V[j] * (1.0 / m[i] + 1.0 / m[j])
        KE[3 * i:3 * i + 3, b] = g * Mb
        KE[3 * j:3 * j + 3, b] = -g * Mb
    return dict(CE=CE, CTH=CTH, KTH=KTH, KE=KE, bi=bi, bj=bj, x=x, M=M, m=m)


def internal_force_operator(w, rho_bond=None, bonds=None):
    """F_int = (K^v + K^d) U as a dense 3N x 3N matrix (Eq. 2.14)."""
    mats = matrices(w, rho_bond, bonds)
    Kv = mats["KTH"] @ mats["CTH"] @ mats["CE"]
    Kd = mats["KE"] @ mats["CE"]
    return Kv + Kd, mats


def mass_vector(w):
    """Diagonal of the lumped mass matrix, 3 entries per node (rho V)."""
    rho = np.array([w.materials[s].rho for s in w.specimen])
    return np.repeat(rho * np.asarray(w.vol), 3)


def free_dofs(w):
    """Indices of the unconstrained degrees of freedom (active components only)."""
    idx = []
    for p in range(w.n):
        for c in range(w.dim):
            if not (int(w.bc[p]) >> c) & 1:
                idx.append(3 * p + c)
    return np.array(idx, dtype=np.int64)


def factored_run(w, nsteps, u, v, s0, dt, rho_bond=None, step0=0, rebuild_ktheta=True):
    """The paper's matrix-based solver loop (Appendix B) on the four global
    matrices, advancing (u, v) in place (n x 3 arrays) by nsteps steps.

    Reading of the failure block, which the listing elides: every intact
    bond whose stretch E_b / x_b (Eq. 1.17, E from C_e U) reaches s0 breaks
    for good (Eq. 1.30) before the dilatation of the same step; a broken
    bond's E_b is zeroed, which removes it from C_theta E and K_e E, and
    K_theta, which does not act through E, is rebuilt for the new bond
    status.  rebuild_ktheta=False keeps K_theta of the initial status (the
    reading in which breaking only masks E; the tests use it to show that it
    is not the loop form).  Returns the bond status (order of
    bonds_bruteforce)."""
    import scipy.sparse as sparse

    intact = matrices(w)
    x = intact["x"]
    nb = len(x)
    rho = np.ones(nb) if rho_bond is None else np.asarray(rho_bond, dtype=np.float64).copy()
    CE = sparse.csr_matrix(intact["CE"])
    CTH = sparse.csr_matrix(intact["CTH"])
    KE = sparse.csr_matrix(intact["KE"])
    KTH = sparse.csr_matrix(matrices(w, rho_bond=rho)["KTH"])
    M = mass_vector(w)
    fixed = np.zeros(3 * w.n, dtype=bool)
    for p in range(w.n):
        for c in range(3):
            fixed[3 * p + c] = bool((int(w.bc[p]) >> c) & 1)
    fext = np.asarray(w.fext, dtype=np.float64).reshape(-1)
    s0b = np.array([s0[w.specimen[i]] for i in intact["bi"]])
    U = u.reshape(-1)
    VEL = v.reshape(-1)
    for it in range(nsteps):
        n = step0 + it
        r = 1.0 if w.ramp_steps <= 0 else min(1.0, n / w.ramp_steps)
        E = CE @ U
        newly = (rho == 1) & (E / x >= s0b)
        if newly.any():
            rho[newly] = 0
            if rebuild_ktheta:
                KTH = sparse.csr_matrix(matrices(w, rho_bond=rho)["KTH"])
        E = E * rho
        Theta = CTH @ E
        PDF = KTH @ Theta + KE @ E
        ACC = (PDF + fext * r) / M
        ACC[fixed] = 0.0
        VEL += dt * ACC
        U += dt * VEL
    return rho.astype(np.uint8)


def sparse_operator(w, o, rho_bond=None):
    """F_int = (K^v + K^d) U (Eq. 2.14) as a scipy sparse matrix, 3N x 3N,
    assembled from the same per-bond blocks as matrices() (Eqs. 2.7-2.10)
    for larger grids: the bonds, bond geometry and weighted volumes come
    from the loop reference o.  A broken bond contributes to none of the
    four matrices."""
    import scipy.sparse as sparse

    bi, bj = o.bonds()
    x, M = o.bond_geom()
    m = o.m()
    n, nb = w.n, len(bi)
    V = np.asarray(w.vol, dtype=np.float64)
    rho = np.ones(nb) if rho_bond is None else np.asarray(rho_bond, dtype=np.float64)
    spec = np.asarray(w.specimen)[bi]
    A = np.empty(nb)
    Kc = np.empty(nb)
    G = np.empty(nb)
    for k, mat in enumerate(w.materials):
        c = constants(w.mode_id(), mat.E, mat.nu)
        sel = spec == k
        A[sel], Kc[sel], G[sel] = c["A"], c["K"], c["G"]
    b = np.arange(nb)
    comp = np.arange(3)
    # Eq. 2.7
    rows = np.repeat(b, 6)
    cols = np.concatenate([3 * bi[:, None] + comp, 3 * bj[:, None] + comp], axis=1).ravel()
    vals = (np.concatenate([-M, M], axis=1) * rho[:, None]).ravel()
    CE = sparse.csr_matrix((vals, (rows, cols)), shape=(nb, 3 * n))
    # Eq. 2.10
    CTH = sparse.csr_matrix((np.concatenate([A * x * V[bj] / m[bi], A * x * V[bi] / m[bj]]) * np.tile(rho, 2),
                             (np.concatenate([bi, bj]), np.concatenate([b, b]))), shape=(n, nb))
    # Eq. 2.8
    cb = (Kc - G / 3.0) * x * V[bi] * V[bj] * rho
    r8, c8, v8 = [], [], []
    for node_row, sgn in ((bi, 1.0), (bj, -1.0)):
        for node_col, mcol in ((bi, m[bi]), (bj, m[bj])):
            r8.append(3 * node_row[:, None] + comp)
            c8.append(np.repeat(node_col[:, None], 3, axis=1))
            v8.append(sgn * (cb / mcol)[:, None] * M)
    KTH = sparse.csr_matrix((np.concatenate(v8).ravel(), (np.concatenate(r8).ravel(), np.concatenate(c8).ravel())),
                            shape=(3 * n, n))
    # Eq. 2.9
    g = G * V[bi] * V[bj] * (1.0 / m[bi] + 1.0 / m[bj]) * rho
    KE = sparse.csr_matrix((np.concatenate([g[:, None] * M, -g[:, None] * M]).ravel(),
                            (np.concatenate([3 * bi[:, None] + comp, 3 * bj[:, None] + comp]).ravel(),
                             np.concatenate([np.repeat(b[:, None], 3, axis=1)] * 2).ravel())),
                           shape=(3 * n, nb))
    return (KTH @ (CTH @ CE) + KE @ CE).tocsr()


def static_solution(w, o, u0=None, rho_bond=None):
    """Static equilibrium F_int(u) + F_ext = 0 on the free components, the
    prescribed components held at their values in u0 (zero if None): a
    direct sparse solve of K_ff du_f = F_ext,f + F_int(u0)_f with K = -F_int'
    (Eq. 2.14).  Returns u (n x 3)."""
    import scipy.sparse.linalg as spla

    L = sparse_operator(w, o, rho_bond)
    u = np.zeros(3 * w.n) if u0 is None else np.asarray(u0, dtype=np.float64).reshape(-1).copy()
    free = free_dofs(w)
    b = np.asarray(w.fext, dtype=np.float64).reshape(-1) + L @ u
    Kff = (-L)[free][:, free].tocsc()
    u[free] += spla.spsolve(Kff, b[free])
    return u.reshape(w.n, 3)


def newmark_run(w, o, u, v, dt, nsteps, rho_bond=None, breaking=False):
    """Implicit dynamics by the average-acceleration Newmark rule (beta = 1/4,
    gamma = 1/2) with the lumped mass rho V and the stiffness of Eq. 2.14.
    Per step, from (u_n, v_n):

    * with ``breaking``, the critical-stretch test of Eqs. 1.17, 1.30 at u_n
      (linearized extension (M1 eta1 + M2 eta2) + M3 eta3 over x >= s_c)
      takes broken bonds out of the operator;
    * a_n from the equation of motion M a_n = F_ext + F_int(u_n) on the free
      components;
    * u* = u_n with the prescribed components advanced by dt v_n;
    * a direct sparse solve of (K_ff + 4/dt^2 M_ff) du_f =
      F_ext + F_int(u*) + M (4 v_n / dt + a_n) on the free components;
    * u_{n+1} = u* + du, a_{n+1} = 4/dt^2 (du - dt v_n) - a_n and
      v_{n+1} = v_n + dt/2 (a_n + a_{n+1}) on the free components.

    Returns (u, v, rho_bond); u and v are n x 3."""
    import scipy.sparse as sparse
    import scipy.sparse.linalg as spla

    u = np.asarray(u, dtype=np.float64).reshape(-1).copy()
    v = np.asarray(v, dtype=np.float64).reshape(-1).copy()
    rho = (o.rho() if rho_bond is None else np.asarray(rho_bond)).astype(np.float64).copy()
    free = free_dofs(w)
    pres = np.array([3 * p + c for p in range(w.n) for c in range(w.dim) if (int(w.bc[p]) >> c) & 1],
                    dtype=np.int64)
    mass = mass_vector(w)
    F = np.asarray(w.fext, dtype=np.float64).reshape(-1)
    k = 4.0 / (dt * dt)
    bi, bj = o.bonds()
    x, M = o.bond_geom()
    s0 = np.asarray(o.s0)[np.asarray(w.specimen)[bi]]
    for _ in range(nsteps):
        if breaking:
            U = u.reshape(-1, 3)
            eta = U[bj] - U[bi]
            e = (M[:, 0] * eta[:, 0] + M[:, 1] * eta[:, 1]) + M[:, 2] * eta[:, 2]
            rho[(rho > 0) & (e / x >= s0)] = 0.0
        L = sparse_operator(w, o, rho)
        a = np.zeros_like(u)
        a[free] = (F + L @ u)[free] / mass[free]
        us = u.copy()
        us[pres] += dt * v[pres]
        b = F + L @ us + mass * (4.0 / dt * v + a)
        Aff = ((-L) + sparse.diags(k * mass))[free][:, free].tocsc()
        du = spla.spsolve(Aff, b[free])
        u = us
        u[free] += du
        a_new = k * (du - dt * v[free]) - a[free]
        v[free] = v[free] + 0.5 * dt * (a[free] + a_new)
    return u.reshape(w.n, 3), v.reshape(w.n, 3), rho
