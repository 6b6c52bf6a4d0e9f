"""Physics-shaped inputs: the Jacobian of an implicit first-order
finite-volume step for a multi-species calorically perfect gas with an HLL
flux, split into the block r1-sparse layout.

This module only builds inputs (it holds none of the linear-algebra path:
no matvec, factorisation or solve).  It follows the paper's setting:

* conserved variables u = (rho_k, rho u, rho v, rho e_tot) and primitive
  solution variables q = (rho_k, u, v, T) (section 2, "Compressible Flow
  Model"; section 3, "Solution Representation"), m = L + 3 with L species;
* the HLL numerical flux written with the scalar coefficients a_f, c_f
  (section 3, eq. HLL_flux; section 4, eq. HLL_flux_compact), the wave-speed
  bounds from (u_n, a) of both sides;
* the trace-flux Jacobians split into a sparse part and two rank-one terms
  (section 4, eqs. r1_flux_left / r1_flux_right), with the sparse parts
  built from H = du/dq and A_n = df_n/dq, both sparse in q.

Gas: species k has the gas constant r_k = 1/M_k, energy e_k(T) = cv_k T +
e0_k (calorically perfect), nondimensional units (reference molar mass,
temperature and density 1).  Species 0..L-2 are levels of one diatomic
species (M = 1, cv = 5/2 r, level energies e0 = 0.3 j r), species L-1 is its
atom (M = 1/2, cv = 3/2 r, e0 = 4 r).  Structured nx x ny mesh of unit
cells, outward unit normals, far-field state on the boundary faces, local
time step dt = cfl / (|u| + |v| + 2 a) frozen in the Jacobian.

Residual of cell c (conservative form with outward normals):
    R_c(Q) = u(q_c) - u(q_c^n) + dt_c sum_faces f_hat(q_c, q_nb, n).
Its Jacobian blocks in the library's layout:
* diagonal block: sparse part H_c + dt_c sum_f [(1/2 + a_f) A_n(q_c) -
  c_f H_c] (diagonal, level rows x flow columns, flow rows x levels, 3 x 3
  corner: the `arrow` pattern with no level band), plus two rank-one pairs
  per face, -(f_nR - f_nL) (da_f/dq_L)^T and (u_R - u_L) (dc_f/dq_L)^T scaled
  by dt_c: r_diag = 8;
* neighbour block: dt_c [(1/2 - a_f) A_n(q_nb) + c_f H_nb] plus the two flux
  pairs with d/dq_R.  Its sparse part is not diagonal (level rows x
  velocity columns, flow rows x everything); the library's neighbour blocks
  keep a diagonal sparse part, so the rest becomes four more exact rank-one
  pairs: (1/2 - a_f) rho_k (levels) x (n_x e_u + n_y e_v), and one pair per
  flow row (unit vector x the row without its diagonal): r_off = 6.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from .gen import DIR_C, DIR_E, DIR_N, DIR_S, DIR_W, NBR_DIRS, pair_slots

# outward unit normal of each face direction
NORMALS = {DIR_S: (0.0, -1.0), DIR_W: (-1.0, 0.0), DIR_E: (1.0, 0.0), DIR_N: (0.0, 1.0)}
FACE_DIRS = (DIR_S, DIR_W, DIR_E, DIR_N)
R_DIAG, R_OFF = 8, 6


def gas(L: int):
    """r_k, cv_k, e0_k of the L species."""
    M = np.ones(L)
    M[-1] = 0.5
    r = 1.0 / M
    cv = 2.5 * r
    cv[-1] = 1.5 * r[-1]
    e0 = 0.3 * np.arange(L) * r
    e0[-1] = 4.0 * r[-1]
    return r, cv, e0


# ---------------------------------------------------- state functions ----
def _split(q, L):
    return q[..., :L], q[..., L], q[..., L + 1], q[..., L + 2]


def conserved(q, L, g):
    r, cv, e0 = g
    rk, u, v, T = _split(q, L)
    rho = rk.sum(-1)
    rhoE = (rk * (cv * T[..., None] + e0)).sum(-1) + 0.5 * rho * (u * u + v * v)
    return np.concatenate([rk, (rho * u)[..., None], (rho * v)[..., None], rhoE[..., None]], -1)


def flux_n(q, n, L, g):
    r, cv, e0 = g
    rk, u, v, T = _split(q, L)
    rho = rk.sum(-1)
    p = (rk * r).sum(-1) * T
    un = n[0] * u + n[1] * v
    rhoE = (rk * (cv * T[..., None] + e0)).sum(-1) + 0.5 * rho * (u * u + v * v)
    return np.concatenate([rk * un[..., None], (rho * u * un + p * n[0])[..., None],
                           (rho * v * un + p * n[1])[..., None], ((rhoE + p) * un)[..., None]], -1)


def sound_speed(q, L, g):
    r, cv, e0 = g
    rk, u, v, T = _split(q, L)
    rho = rk.sum(-1)
    Scv, Sr = (rk * cv).sum(-1), (rk * r).sum(-1)
    return np.sqrt((Scv + Sr) * Sr * T / (Scv * rho))


# H and A_n are nonzero only on the level diagonal, in the level rows x flow
# columns and in the three flow rows; a "parts" triple holds exactly those:
# (level diagonal [..., L], level x flow [..., L, 3], flow rows [..., 3, m]).
def dense(parts, L):
    """The m x m matrices of a parts triple."""
    lev, lf, fr = parts
    m = L + 3
    X = np.zeros(np.shape(lev)[:-1] + (m, m))
    k = np.arange(L)
    X[..., k, k] = lev
    X[..., :L, L:] = lf
    X[..., L:, :] = fr
    return X


def combine(terms):
    """sum_i c_i X_i over (c_i [...], parts_i) on the parts triples."""
    out = None
    for c, (lev, lf, fr) in terms:
        c = np.asarray(c)[..., None]
        t = (c * lev, c[..., None] * lf, c[..., None] * fr)
        out = t if out is None else tuple(a + b for a, b in zip(out, t))
    return out


def H_parts(q, L, g):
    """du/dq for states q [..., m], as a parts triple."""
    r, cv, e0 = g
    rk, u, v, T = _split(q, L)
    m = L + 3
    rho = rk.sum(-1)
    lev = np.ones(np.shape(rk))
    lf = np.zeros(np.shape(rk) + (3,))
    fr = np.zeros(np.shape(q)[:-1] + (3, m))
    fr[..., 0, :L] = u[..., None]
    fr[..., 0, L] = rho
    fr[..., 1, :L] = v[..., None]
    fr[..., 1, L + 1] = rho
    fr[..., 2, :L] = cv * T[..., None] + e0 + 0.5 * (u * u + v * v)[..., None]
    fr[..., 2, L] = rho * u
    fr[..., 2, L + 1] = rho * v
    fr[..., 2, L + 2] = (rk * cv).sum(-1)
    return lev, lf, fr


def A_parts(q, n, L, g):
    """df_n/dq for states q [..., m] and the normal n, as a parts triple."""
    r, cv, e0 = g
    rk, u, v, T = _split(q, L)
    m = L + 3
    rho = rk.sum(-1)
    Sr, Scv = (rk * r).sum(-1), (rk * cv).sum(-1)
    un = n[0] * u + n[1] * v
    ek = cv * T[..., None] + e0 + 0.5 * (u * u + v * v)[..., None]
    rhoE = (rk * (cv * T[..., None] + e0)).sum(-1) + 0.5 * rho * (u * u + v * v)
    p = Sr * T
    lev = un[..., None] * np.ones(np.shape(rk))
    lf = np.zeros(np.shape(rk) + (3,))
    lf[..., 0] = rk * n[0]
    lf[..., 1] = rk * n[1]
    fr = np.zeros(np.shape(q)[:-1] + (3, m))
    fr[..., 0, :L] = (u * un)[..., None] + r * T[..., None] * n[0]
    fr[..., 0, L] = rho * (un + u * n[0])
    fr[..., 0, L + 1] = rho * u * n[1]
    fr[..., 0, L + 2] = Sr * n[0]
    fr[..., 1, :L] = (v * un)[..., None] + r * T[..., None] * n[1]
    fr[..., 1, L] = rho * v * n[0]
    fr[..., 1, L + 1] = rho * (un + v * n[1])
    fr[..., 1, L + 2] = Sr * n[1]
    fr[..., 2, :L] = (ek + r * T[..., None]) * un[..., None]
    fr[..., 2, L] = rho * u * un + (rhoE + p) * n[0]
    fr[..., 2, L + 1] = rho * v * un + (rhoE + p) * n[1]
    fr[..., 2, L + 2] = (Scv + Sr) * un
    return lev, lf, fr


def H_matrix(q, L, g):
    """du/dq for states q [..., m] (one dense matrix per state)."""
    return dense(H_parts(q, L, g), L)


def A_matrix(q, n, L, g):
    """df_n/dq for states q [..., m] and the normal n (dense)."""
    return dense(A_parts(q, n, L, g), L)


def grad_sound_speed(q, L, g):
    """da/dq for states q [..., m]."""
    r, cv, e0 = g
    rk, u, v, T = _split(q, L)
    rho = rk.sum(-1)
    Scv, Sr = (rk * cv).sum(-1), (rk * r).sum(-1)
    a2 = (Scv + Sr) * Sr * T / (Scv * rho)
    a = np.sqrt(a2)
    da2 = np.zeros(np.shape(q))
    Scv_, Sr_, rho_, T_ = Scv[..., None], Sr[..., None], rho[..., None], T[..., None]
    da2[..., :L] = T_ * ((cv + r) * Sr_ / (Scv_ * rho_) + (Scv_ + Sr_) * r / (Scv_ * rho_)
                         - (Scv_ + Sr_) * Sr_ * cv / (Scv_ * Scv_ * rho_)
                         - (Scv_ + Sr_) * Sr_ / (Scv_ * rho_ * rho_))
    da2[..., L + 2] = a2 / T
    return da2 / (2.0 * a[..., None])


# ------------------------------------------------- DRa source (optional) ----
# Dissociation and recombination of the molecule levels by atom impact
# (section 4, "Temporal Source Jacobian": each level's rate depends on its own
# density, the atom density and the temperature; the atom's on every level).
# Toy Arrhenius-like rates, level v = 0..L-2, atom a = L-1:
#   Omega_v = -kd_v(T) rho_v rho_a + kr_v(T) rho_a^3,   Omega_a = -sum_v Omega_v
#   kd_v = DRA_KD exp(-theta_v / T), theta_v = DRA_THETA (1 - v / (L-1)),
#   kr_v = DRA_KR exp(-0.1 v) / T.
DRA_KD, DRA_THETA, DRA_KR = 20.0, 3.0, 200.0


def dra_rates(T, L):
    """kd, kr [..., L-1] and their T-derivatives at temperatures T [...]."""
    v = np.arange(L - 1)
    theta = DRA_THETA * (1.0 - v / (L - 1))
    T_ = np.asarray(T)[..., None]
    kd = DRA_KD * np.exp(-theta / T_)
    kr = DRA_KR * np.exp(-0.1 * v) / T_
    return kd, kr, kd * theta / (T_ * T_), -kr / T_


def dra_source(q, L):
    """Omega [..., m] (zero in the flow rows: the source moves mass between
    species and leaves momentum and total energy unchanged)."""
    rk, T = q[..., :L], q[..., L + 2]
    kd, kr, _, _ = dra_rates(T, L)
    ra = rk[..., L - 1:L]
    om = np.zeros(np.shape(q))
    om[..., :L - 1] = -kd * rk[..., :L - 1] * ra + kr * ra ** 3
    om[..., L - 1] = -om[..., :L - 1].sum(-1)
    return om


def dra_parts(q, L):
    """dOmega/dq as its nonzero pieces: level diagonal [..., L], the T column
    [..., L], the atom column over the molecule levels [..., L-1] and the
    atom row over them [..., L-1]."""
    rk, T = q[..., :L], q[..., L + 2]
    kd, kr, dkd, dkr = dra_rates(T, L)
    rv, ra = rk[..., :L - 1], rk[..., L - 1:L]
    diag = np.zeros(np.shape(rk))
    diag[..., :L - 1] = -kd * ra
    col = -kd * rv + 3.0 * kr * ra * ra
    diag[..., L - 1] = -col.sum(-1)
    tcol = np.zeros(np.shape(rk))
    tcol[..., :L - 1] = -dkd * rv * ra + dkr * ra ** 3
    tcol[..., L - 1] = -tcol[..., :L - 1].sum(-1)
    row = kd * ra
    return diag, tcol, col, row


# ------------------------------------------------------------ HLL flux ----
def hll(qL, qR, n, L, g):
    """HLL flux and its pieces for states [..., m]: f_hat, a_f, c_f, and
    da_f, dc_f w.r.t. qL and qR (wave-speed bounds s_L = min(u_nL - a_L,
    u_nR - a_R), s_R = max(u_nL + a_L, u_nR + a_R), the branch taken at
    ties: left)."""
    m = L + 3
    aL, aR = sound_speed(qL, L, g), sound_speed(qR, L, g)
    unL = n[0] * qL[..., L] + n[1] * qL[..., L + 1]
    unR = n[0] * qR[..., L] + n[1] * qR[..., L + 1]
    dun = np.zeros(m)
    dun[L], dun[L + 1] = n
    daL, daR = grad_sound_speed(qL, L, g), grad_sound_speed(qR, L, g)
    zero = np.zeros(np.shape(daL))
    left_lo = (unL - aL <= unR - aR)[..., None]
    left_hi = (unL + aL >= unR + aR)[..., None]
    sL = np.where(left_lo[..., 0], unL - aL, unR - aR)
    dsL_L = np.where(left_lo, dun - daL, zero)
    dsL_R = np.where(left_lo, zero, dun - daR)
    sR = np.where(left_hi[..., 0], unL + aL, unR + aR)
    dsR_L = np.where(left_hi, dun + daL, zero)
    dsR_R = np.where(left_hi, zero, dun + daR)
    D = sR - sL
    af = 0.5 * (sL + sR) / D
    cf = sL * sR / D
    # a_f = (s_L + s_R) / (2 (s_R - s_L)):  da_f = (s_R ds_L - s_L ds_R) / D^2
    # c_f = s_L s_R / (s_R - s_L):          dc_f = (s_R^2 ds_L - s_L^2 ds_R) / D^2
    sL_, sR_, D2 = sL[..., None], sR[..., None], (D * D)[..., None]
    daf_L = (sR_ * dsL_L - sL_ * dsR_L) / D2
    daf_R = (sR_ * dsL_R - sL_ * dsR_R) / D2
    dcf_L = (sR_ * sR_ * dsL_L - sL_ * sL_ * dsR_L) / D2
    dcf_R = (sR_ * sR_ * dsL_R - sL_ * sL_ * dsR_R) / D2
    fL, fR = flux_n(qL, n, L, g), flux_n(qR, n, L, g)
    uL, uR = conserved(qL, L, g), conserved(qR, L, g)
    fhat = (0.5 * (fL + fR) - af[..., None] * (fR - fL) + cf[..., None] * (uR - uL))
    return dict(fhat=fhat, af=af, cf=cf, daf_L=daf_L, daf_R=daf_R, dcf_L=dcf_L, dcf_R=dcf_R,
                fL=fL, fR=fR, uL=uL, uR=uR)


# ---------------------------------------------------------------- state ----
def make_state(nx: int, ny: int, L: int, seed: int = 0, cfl: float = 1.0):
    """A smooth subsonic state on the mesh, the far-field state and the
    local time steps: {"q": [N][m], "q_inf": [m], "dt": [N]}."""
    rng = np.random.default_rng(seed)
    N = nx * ny
    iy, ix = np.divmod(np.arange(N), nx)
    X, Y = (ix + 0.5) / nx, (iy + 0.5) / ny
    # Boltzmann-like level populations, a few percent atoms, smooth waves
    lev = np.exp(-0.4 * np.arange(L - 1)) if L > 1 else np.zeros(0)
    base = np.concatenate([lev / max(lev.sum(), 1e-300) * 0.95, [0.05]]) if L > 1 else np.ones(1)
    wave = 1.0 + 0.1 * np.sin(2 * np.pi * X)[:, None] * np.cos(2 * np.pi * Y)[:, None]
    rk = base[None, :] * wave * (1.0 + 0.05 * rng.standard_normal((N, L)))
    u = 0.3 + 0.05 * np.sin(2 * np.pi * Y) + 0.02 * rng.standard_normal(N)
    v = 0.1 * np.sin(2 * np.pi * X) + 0.02 * rng.standard_normal(N)
    T = 1.0 + 0.1 * np.cos(2 * np.pi * X) + 0.02 * rng.standard_normal(N)
    q = np.concatenate([rk, u[:, None], v[:, None], T[:, None]], 1)
    q_inf = np.concatenate([base, [0.3, 0.0, 1.0]])
    g = gas(L)
    a = sound_speed(q, L, g)
    dt = cfl / (np.abs(u) + np.abs(v) + 2.0 * a)
    return {"q": q, "q_inf": q_inf, "dt": dt}


def _neighbours(nx, ny, d):
    """Neighbour of every cell across face direction d (-1 on the boundary)."""
    c = np.arange(nx * ny)
    iy, ix = np.divmod(c, nx)
    if d == DIR_S:
        return np.where(iy > 0, c - nx, -1)
    if d == DIR_W:
        return np.where(ix > 0, c - 1, -1)
    if d == DIR_E:
        return np.where(ix < nx - 1, c + 1, -1)
    return np.where(iy < ny - 1, c + nx, -1)


def _right_states(Q, q_inf, nb):
    """The state across each face: the neighbour's, or the far field."""
    return np.where((nb >= 0)[:, None], Q[np.maximum(nb, 0)], q_inf)


def residual(st, nx: int, ny: int, L: int, Q=None, u_old=None, dra: bool = False):
    """R_c(Q) = u(q_c) - u_old_c + dt_c sum_faces f_hat (dt frozen), and
    - dt_c Omega(q_c) with the DRa source; with the defaults Q is the state
    and u_old its conserved variables (R = flux part only)."""
    g = gas(L)
    Q = st["q"] if Q is None else Q
    R = conserved(Q, L, g) - (conserved(st["q"], L, g) if u_old is None else u_old)
    for d in FACE_DIRS:
        qR = _right_states(Q, st["q_inf"], _neighbours(nx, ny, d))
        R = R + st["dt"][:, None] * hll(Q, qR, NORMALS[d], L, g)["fhat"]
    if dra:
        R = R - st["dt"][:, None] * dra_source(Q, L)
    return R


CHUNK = 1024  # cells per batch in make_problem (bounds the m x m temporaries)


def make_problem(nx: int, ny: int, L: int, seed: int = 0, cfl: float = 1.0,
                 dra: bool = False) -> Dict[str, np.ndarray]:
    """The Jacobian dR/dQ at the state, in the library's structured layout
    with 8 pairs per diagonal block, 6 per neighbour block, no level band and
    level/flow coupling (see the module docstring).  With the DRa source the
    pattern is arrow = 2: its atom column and row go to slot 3 of s_lev_flow
    and s_flow_lev, its diagonal and T column to s_diag and slot 2."""
    if L < 2:
        raise ValueError("need at least two species")
    st = make_state(nx, ny, L, seed, cfl)
    g = gas(L)
    N, m = nx * ny, L + 3
    P = R_DIAG + 4 * R_OFF
    slots = pair_slots(R_DIAG, R_OFF)
    p = {k: np.zeros(s) for k, s in (("s_diag", (N, m)), ("s_sub", (N, L - 1)),
                                      ("s_sup", (N, L - 1)), ("s_flow", (N, 6)),
                                      ("s_nbr", (N, 4, m)), ("u", (N, P, m)), ("v", (N, P, m)),
                                      ("s_band", (N, 0, L)), ("s_lev_flow", (N, 3 + dra, L)),
                                      ("s_flow_lev", (N, 3 + dra, L)))}
    corner = ((0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1))
    nbrs = {d: _neighbours(nx, ny, d) for d in FACE_DIRS}
    a0 = slots[DIR_C][0]
    u, v = p["u"], p["v"]
    for c0 in range(0, N, CHUNK):
        cs = slice(c0, min(N, c0 + CHUNK))
        qc, dt = st["q"][cs], st["dt"][cs]
        Hc = H_parts(qc, L, g)
        S = [(np.ones_like(dt), Hc)]
        for t, d in enumerate(FACE_DIRS):
            n = NORMALS[d]
            nb = nbrs[d][cs]
            inside = nb >= 0
            qR = _right_states(st["q"], st["q_inf"], nb)
            h = hll(qc, qR, n, L, g)
            af, cf = h["af"], h["cf"]
            S += [(dt * (0.5 + af), A_parts(qc, n, L, g)), (-dt * cf, Hc)]
            dt2 = dt[:, None]
            # the two flux pairs of the diagonal block (d/dq_L)
            u[cs, a0 + 2 * t] = -dt2 * (h["fR"] - h["fL"])
            v[cs, a0 + 2 * t] = h["daf_L"]
            u[cs, a0 + 2 * t + 1] = dt2 * (h["uR"] - h["uL"])
            v[cs, a0 + 2 * t + 1] = h["dcf_L"]
            # neighbour block (interior faces only): dt [(1/2 - a_f) A_n(q_nb)
            # + c_f H_nb] + flux pairs
            w = np.where(inside, dt, 0.0)
            glev, glf, gfr = combine([(w * (0.5 - af), A_parts(qR, n, L, g)),
                                      (w * cf, H_parts(qR, L, g))])
            j = NBR_DIRS.index(d)
            p["s_nbr"][cs, j, :L] = glev
            for i in range(3):
                p["s_nbr"][cs, j, L + i] = gfr[:, i, L + i]
            a = slots[d][0]
            ins = inside[:, None]
            u[cs, a] = np.where(ins, -dt2 * (h["fR"] - h["fL"]), 0.0)
            v[cs, a] = np.where(ins, h["daf_R"], 0.0)
            u[cs, a + 1] = np.where(ins, dt2 * (h["uR"] - h["uL"]), 0.0)
            v[cs, a + 1] = np.where(ins, h["dcf_R"], 0.0)
            # level rows x velocity columns: dt (1/2 - a_f) rho_k (n_x e_u + n_y e_v)
            u[cs, a + 2, :L] = (w * (0.5 - af))[:, None] * qR[:, :L]
            v[cs, a + 2, L] = np.where(inside, n[0], 0.0)
            v[cs, a + 2, L + 1] = np.where(inside, n[1], 0.0)
            # flow rows without their diagonal entries
            for i in range(3):
                u[cs, a + 3 + i, L + i] = inside
                row = gfr[:, i].copy()
                row[:, L + i] = 0.0
                v[cs, a + 3 + i] = row
        slev, slf, sfr = combine(S)
        p["s_diag"][cs, :L] = slev
        for i in range(3):
            p["s_diag"][cs, L + i] = sfr[:, i, L + i]
        p["s_lev_flow"][cs, :3] = slf.transpose(0, 2, 1)
        p["s_flow_lev"][cs, :3] = sfr[:, :, :L]
        for t, (i, j) in enumerate(corner):
            p["s_flow"][cs, t] = sfr[:, i, L + j]
        if dra:
            sd, tcol, col, row = dra_parts(qc, L)
            w = -dt[:, None]
            p["s_diag"][cs, :L] += w * sd
            p["s_lev_flow"][cs, 2] += w * tcol
            p["s_lev_flow"][cs, 3, :L - 1] = w * col
            p["s_flow_lev"][cs, 3, :L - 1] = w * row
    for k in list(p):
        p[k] = np.ascontiguousarray(p[k])
    p["ranks"] = np.array([R_DIAG, R_OFF])
    p["pattern"] = np.array([1, 2 if dra else 1])
    p["state"] = st["q"]
    return p
