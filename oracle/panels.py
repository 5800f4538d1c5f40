"""Panel extraction from a voxel grid (oracle).

Follows Sec. II.A (eq. 3) and the voxel-panel description of Sec. II.B: the
charge unknowns live on unit-square faces of the voxel grid.  A face carries a
conductor panel when exactly one of its two voxels is a conductor, and a
dielectric panel when neither is and their permittivities differ.  Faces on the
grid boundary see the background medium (permittivity eps_b) outside.

Dielectric panels use the paper's orientation (eq. 2): the unit normal points
out of the dielectric, i.e. from the side of larger permittivity (eps_d) into
the side of smaller permittivity (eps_b); `sign` is +1 when that normal is the
+axis direction and -1 when it is the -axis direction (Sec. II.B, note 3).
"""
from __future__ import annotations

import numpy as np


class GeometryError(ValueError):
    pass


def panelize(cond_id, eps_r, eps_b=1.0):
    """Return a dict of panel arrays, in the oracle's own order (axis, then grid index).

    axis[k]   normal axis (0=x, 1=y, 2=z)
    idx[k]    (i, j, k) grid index; the face lies at coordinate idx[axis] along axis
              and spans [idx, idx+1] along the other two axes
    center[k] face centre in voxel units
    kind[k]   0 conductor, 1 dielectric
    cond[k]   conductor id (conductor panels), -1 otherwise
    eps_adj[k]  relative permittivity next to a conductor panel
    eps_d, eps_b_side, sign  dielectric panels (paper convention, see module doc)
    eps_lo, eps_hi  permittivity on the -axis / +axis side (all panels)
    """
    cond_id = np.asarray(cond_id)
    eps_r = np.asarray(eps_r, dtype=np.float64)
    if cond_id.shape != eps_r.shape or cond_id.ndim != 3:
        raise GeometryError("cond_id and eps_r must be equal 3-D shapes")
    if np.any((cond_id < 0) & ~(eps_r > 0)):
        raise GeometryError("non-positive permittivity")
    if eps_b <= 0:
        raise GeometryError("non-positive background permittivity")
    if not np.any(cond_id >= 0):
        raise GeometryError("no conductor")
    out = {k: [] for k in ("axis", "idx", "kind", "cond", "eps_adj", "eps_lo", "eps_hi")}
    for a in range(3):
        # pad along axis a with one background voxel on each side
        pad = [(0, 0)] * 3
        pad[a] = (1, 1)
        c = np.pad(cond_id, pad, constant_values=-1)
        e = np.pad(eps_r, pad, constant_values=eps_b)
        e = np.where(c >= 0, np.nan, e)
        n = cond_id.shape[a]
        lo_c = np.take(c, np.arange(0, n + 1), axis=a)
        hi_c = np.take(c, np.arange(1, n + 2), axis=a)
        lo_e = np.take(e, np.arange(0, n + 1), axis=a)
        hi_e = np.take(e, np.arange(1, n + 2), axis=a)
        lo_is = lo_c >= 0
        hi_is = hi_c >= 0
        if np.any(lo_is & hi_is & (lo_c != hi_c)):
            raise GeometryError("two different conductors share a face")
        condf = lo_is ^ hi_is
        dielf = (~lo_is) & (~hi_is) & (lo_e != hi_e)
        for kind, mask in ((0, condf), (1, dielf)):
            ii = np.argwhere(mask)
            m = len(ii)
            if m == 0:
                continue
            sel = tuple(ii.T)
            out["axis"].append(np.full(m, a))
            out["idx"].append(ii)
            out["kind"].append(np.full(m, kind))
            if kind == 0:
                cid = np.where(lo_is[sel], lo_c[sel], hi_c[sel])
                adj = np.where(lo_is[sel], hi_e[sel], lo_e[sel])
                out["cond"].append(cid)
                out["eps_adj"].append(adj)
                out["eps_lo"].append(np.where(lo_is[sel], np.nan, lo_e[sel]))
                out["eps_hi"].append(np.where(hi_is[sel], np.nan, hi_e[sel]))
            else:
                out["cond"].append(np.full(m, -1))
                out["eps_adj"].append(np.full(m, np.nan))
                out["eps_lo"].append(lo_e[sel])
                out["eps_hi"].append(hi_e[sel])
    p = {k: np.concatenate(v) if v else np.zeros(0) for k, v in out.items()}
    # stable order: conductor panels first, then dielectric (as in eq. 4), each by axis/index
    key = np.lexsort((p["idx"][:, 2], p["idx"][:, 1], p["idx"][:, 0], p["axis"], p["kind"]))
    p = {k: v[key] for k, v in p.items()}
    p["axis"] = p["axis"].astype(np.int64)
    p["kind"] = p["kind"].astype(np.int64)
    p["cond"] = p["cond"].astype(np.int64)
    p["idx"] = p["idx"].astype(np.int64)
    center = p["idx"].astype(np.float64) + 0.5
    center[np.arange(len(center)), p["axis"]] -= 0.5
    p["center"] = center
    diel = p["kind"] == 1
    lo, hi = p["eps_lo"], p["eps_hi"]
    # paper orientation: normal out of the larger-permittivity side
    p["sign"] = np.where(diel, np.where(lo > hi, 1, -1), 0).astype(np.int64)
    p["eps_d"] = np.where(diel, np.maximum(lo, hi), np.nan)
    p["eps_b_side"] = np.where(diel, np.minimum(lo, hi), np.nan)
    p["n_cond"] = int(np.sum(p["kind"] == 0))
    p["n_diel"] = int(np.sum(diel))
    p["m"] = int(cond_id.max()) + 1
    return p
