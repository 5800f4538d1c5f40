"""Dense Galerkin system, LU solve and capacitance (oracle).

* assemble(): the N x N matrix of eq. (4), rows in the oracle panel order:
  conductor rows hold P of eq. (5); dielectric rows hold E of eq. (6) taken along
  the paper's outward normal (sign * axis, Sec. II.B note 3) plus the diagonal jump
  term of eq. (7), I_kk = 2*pi*(eps_d + eps_b)/(eps_d - eps_b) in units with
  4*pi*eps0 = 1 and unit panel area.  Entries are the plain integrals, looked up
  per (observer axis, source axis, centre offset) so each distinct offset is
  integrated once.
* rhs(): unit potential on one conductor at a time (Sec. II.A, text after eq. 7).
* capacitance(): eq. (8) with the conductor charge scaled by the relative
  permittivity next to each panel (Sec. II.A, last note), in farads:
  C_ij = 4*pi*eps0*dv * sum_{k in conductor i} eps_adj(k) * rho_k^(j).
* capacitance_gradient(): dC/d(eps of voxel blocks) by one adjoint solve per
  conductor: dC_ij = (dW_i)^T rho_j - lambda_i^T (dA) rho_j with A^T lambda_i = W_i.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import integrals
from .panels import panelize

EPS0 = 8.8541878128e-12          # F/m (CODATA 2018)


def _jump(p):
    """Diagonal of eq. (7) for dielectric panels (paper orientation)."""
    ed, eb = p["eps_d"], p["eps_b_side"]
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(p["kind"] == 1, 2.0 * np.pi * (ed + eb) / (ed - eb), 0.0)


def _lag_codes(co, cs):
    """Integer codes of 2*(co - cs) for all pairs (rows x cols)."""
    d2 = np.rint(2.0 * (co[:, None, :] - cs[None, :, :])).astype(np.int64)
    return d2


def _block(A, p, rows, cols, want, row_scale=None, chunk_elems=20_000_000):
    """Fill A[rows, cols] with `want` integrals, integrating each distinct offset once."""
    if len(rows) == 0 or len(cols) == 0:
        return
    alpha = int(p["axis"][rows[0]])
    beta = int(p["axis"][cols[0]])
    co = p["center"][rows]
    cs = p["center"][cols]
    d2_min = np.rint(2 * (co.min(0) - cs.max(0))).astype(np.int64)
    d2_max = np.rint(2 * (co.max(0) - cs.min(0))).astype(np.int64)
    span = d2_max - d2_min + 1
    used = np.zeros(int(np.prod(span)), bool)
    step = max(1, chunk_elems // len(cols))
    def codes(r0):
        d2 = _lag_codes(co[r0:r0 + step], cs) - d2_min
        return (d2[..., 0] * span[1] + d2[..., 1]) * span[2] + d2[..., 2]
    for r0 in range(0, len(rows), step):
        used[codes(r0).ravel()] = True
    uid = np.nonzero(used)[0]
    d2 = np.stack(np.unravel_index(uid, tuple(span)), axis=1) + d2_min
    vals = integrals.kernel(alpha, beta, d2 / 2.0, want)
    table = np.zeros(len(used))
    table[uid] = vals
    for r0 in range(0, len(rows), step):
        blk = table[codes(r0)]
        if row_scale is not None:
            blk = blk * row_scale[r0:r0 + step, None]
        A[np.ix_(rows[r0:r0 + step], cols)] = blk


def assemble(p):
    """Dense matrix of eq. (4) (dimensionless), rows/cols in oracle panel order."""
    n = len(p["axis"])
    A = np.zeros((n, n))
    for a in range(3):
        for kind in (0, 1):
            rows = np.nonzero((p["axis"] == a) & (p["kind"] == kind))[0]
            if len(rows) == 0:
                continue
            scale = None if kind == 0 else p["sign"][rows].astype(np.float64)
            for b in range(3):
                cols = np.nonzero(p["axis"] == b)[0]
                _block(A, p, rows, cols, "P" if kind == 0 else "E", scale)
    A[np.diag_indices(n)] += _jump(p)
    return A


def assemble_rows(p, rows):
    """Rows `rows` (oracle order) of the matrix of eq. (4), with the same integrals and
    row conventions as assemble(), for a bounded sample of a system too large to
    assemble whole.  Every entry is integrated directly from its centre offset, one row
    and source axis at a time (no offset table), so memory stays O(N)."""
    rows = np.asarray(rows, dtype=np.int64)
    n = len(p["axis"])
    A = np.zeros((len(rows), n))
    cols_of = [np.nonzero(p["axis"] == b)[0] for b in range(3)]
    jump = _jump(p)
    for t, k in enumerate(rows):
        alpha = int(p["axis"][k])
        diel = p["kind"][k] == 1
        for b in range(3):
            cols = cols_of[b]
            if len(cols) == 0:
                continue
            d = p["center"][k][None, :] - p["center"][cols]
            v = integrals.kernel(alpha, b, d, "E" if diel else "P")
            A[t, cols] = float(p["sign"][k]) * v if diel else v
        A[t, k] += jump[k]
    return A


def rhs(p):
    """Unit potential on conductor j, zero on the others and on dielectric rows."""
    n = len(p["axis"])
    B = np.zeros((n, p["m"]))
    c = p["kind"] == 0
    B[np.nonzero(c)[0], p["cond"][c]] = 1.0
    return B


def free_charge_weights(p):
    """W[k, i] = eps_adj(k) for conductor panel k of conductor i (Sec. II.A last note)."""
    W = rhs(p)
    W *= np.where(p["kind"] == 0, p["eps_adj"], 0.0)[:, None]
    return W


def mvp(A, x):
    return A @ x


def solve(A, B):
    lu = sla.lu_factor(A)
    return sla.lu_solve(lu, B), lu


def capacitance_from_rho(p, rho, dv):
    W = free_charge_weights(p)
    return 4.0 * np.pi * EPS0 * dv * (W.T @ rho)


def solve_capacitance(scene, return_all=False):
    """Capacitance matrix (F) of a scene dict from the `scenes` generators."""
    p = panelize(scene["cond_id"], scene["eps_r"], scene["eps_b"])
    A = assemble(p)
    rho, lu = solve(A, rhs(p))
    C = capacitance_from_rho(p, rho, scene["dv"])
    if return_all:
        return C, {"panels": p, "A": A, "rho": rho, "lu": lu}
    return C


def _voxel_block(p, shape, block_of_voxel, side):
    """Block id of the voxel on the -axis (side=0) or +axis (side=1) side of each panel."""
    idx = p["idx"].copy()
    ax = p["axis"]
    if side == 0:
        idx[np.arange(len(idx)), ax] -= 1
    inside = np.all((idx >= 0) & (idx < np.asarray(shape)[None, :]), axis=1)
    out = np.full(len(idx), -1, np.int64)
    ii = idx[inside]
    out[inside] = block_of_voxel[ii[:, 0], ii[:, 1], ii[:, 2]]
    return out


def capacitance_gradient(scene, block_of_voxel, nblocks):
    """dC/d(eps_r of block b), shape (nblocks, m, m), in farads per unit eps_r.

    The matrix depends on the permittivities only through the jump term of eq. (7)
    and the free-charge weights of eq. (8)."""
    C, st = solve_capacitance(scene, return_all=True)
    p, rho, lu = st["panels"], st["rho"], st["lu"]
    shape = scene["cond_id"].shape
    W = free_charge_weights(p)
    lam = sla.lu_solve(lu, W, trans=1)              # A^T lambda_i = W_i
    blo = _voxel_block(p, shape, block_of_voxel, 0)
    bhi = _voxel_block(p, shape, block_of_voxel, 1)
    lo, hi = p["eps_lo"], p["eps_hi"]
    diel = p["kind"] == 1
    ed, eb = p["eps_d"], p["eps_b_side"]
    with np.errstate(invalid="ignore", divide="ignore"):
        dI_ded = np.where(diel, -4.0 * np.pi * eb / (ed - eb) ** 2, 0.0)
        dI_deb = np.where(diel, 4.0 * np.pi * ed / (ed - eb) ** 2, 0.0)
    d_is_lo = lo > hi
    bd = np.where(d_is_lo, blo, bhi)       # block of the eps_d side
    bb = np.where(d_is_lo, bhi, blo)       # block of the eps_b side
    cond = p["kind"] == 0
    # block of the non-conductor voxel next to each conductor panel
    lo_is_cond = np.isnan(lo)
    badj = np.where(lo_is_cond, bhi, blo)
    m = p["m"]
    out = np.zeros((nblocks, m, m))
    scale = 4.0 * np.pi * EPS0 * scene["dv"]
    for b in range(nblocks):
        dW = rhs(p) * (cond & (badj == b))[:, None]
        dA = np.zeros(len(lo))
        dA += np.where(diel & (bd == b), dI_ded, 0.0)
        dA += np.where(diel & (bb == b), dI_deb, 0.0)
        out[b] = scale * (dW.T @ rho - lam.T @ (dA[:, None] * rho))
    return out, C
