"""ctypes binding of libvoxcap.so (include/voxcap.h).  Argument marshalling only:
every step of the solve runs in the HIP library.  Device buffers are torch tensors
(PyTorch supplies device memory and streams); host arrays are numpy.

The functions named vc_* mirror the C entry points one to one; `Problem` wraps them.
If the shared library is missing this module raises at import: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvoxcap.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2004_02609_amd/build.py "
                      "(or __graft_entry__.build())")
_lib = C.CDLL(LIB_PATH)

VC_OK, VC_ERR_ARG, VC_ERR_GEOMETRY, VC_ERR_HIP, VC_ERR_OOM, VC_ERR_NOT_CONVERGED, VC_ERR_NUMERIC, VC_ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7
VC_FP64, VC_FP32, VC_MIXED = 0, 1, 2
_PREC = {"fp64": VC_FP64, "fp32": VC_FP32, "mixed": VC_MIXED}


class vc_geometry(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dv", C.c_double),
                ("cond_id", C.POINTER(C.c_int32)), ("eps_r", C.POINTER(C.c_double)),
                ("eps_background", C.c_double)]


class vc_panel(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("k", C.c_int32), ("dir", C.c_int8), ("kind", C.c_int8),
                ("pad", C.c_int16), ("cond", C.c_int32), ("eps_lo", C.c_double), ("eps_hi", C.c_double),
                ("eps_adj", C.c_double)]


PANEL_DTYPE = np.dtype({"names": ["i", "j", "k", "dir", "kind", "pad", "cond", "eps_lo", "eps_hi", "eps_adj"],
                        "formats": ["<i4", "<i4", "<i4", "i1", "i1", "<i2", "<i4", "<f8", "<f8", "<f8"],
                        "offsets": [vc_panel.i.offset, vc_panel.j.offset, vc_panel.k.offset, vc_panel.dir.offset,
                                    vc_panel.kind.offset, vc_panel.pad.offset, vc_panel.cond.offset,
                                    vc_panel.eps_lo.offset, vc_panel.eps_hi.offset, vc_panel.eps_adj.offset],
                        "itemsize": C.sizeof(vc_panel)})


class vc_setup_opts(C.Structure):
    _fields_ = [("fft_size", C.c_int32 * 3), ("nv", C.c_int32 * 3), ("tucker_tol", C.c_double),
                ("precisions", C.c_int32), ("max_rhs", C.c_int32), ("autotune", C.c_int32),
                ("tune_cache", C.c_char_p)]


class vc_solve_opts(C.Structure):
    _fields_ = [("prec", C.c_int), ("rtol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("inner_rtol", C.c_double), ("ir_max", C.c_int32), ("use_precond", C.c_int32),
                ("graph", C.c_int32), ("mixed_form", C.c_int32)]


class vc_stats(C.Structure):
    _fields_ = [("iters", C.c_int32 * 64), ("final_rre", C.c_double * 64), ("ir_steps", C.c_int32),
                ("mvp_count", C.c_int32), ("t_setup_s", C.c_double), ("t_solve_s", C.c_double),
                ("spectra_bytes", C.c_double), ("tucker_rank_max", C.c_int32), ("bytes_model", C.c_double),
                ("mixed_form", C.c_int32), ("steps_fp32", C.c_int32)]


_P = C.c_void_p
_sig = {
    "vc_problem_create": (C.c_int, [C.POINTER(vc_geometry), C.c_int, C.POINTER(_P)]),
    "vc_problem_destroy": (C.c_int, [_P]),
    "vc_panel_counts": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "vc_panels": (C.c_int, [_P, C.c_void_p]),
    "vc_fft_size": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "vc_setup": (C.c_int, [_P, C.POINTER(vc_setup_opts), _P]),
    "vc_apply": (C.c_int, [_P, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int32, _P]),
    "vc_apply_precond": (C.c_int, [_P, C.c_int, C.c_void_p, C.c_void_p, C.c_int32, _P]),
    "vc_apply_precond_kind": (C.c_int, [_P, C.c_int32, C.c_int, C.c_void_p, C.c_void_p, C.c_int32, _P]),
    "vc_precond_info": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "vc_capacitance": (C.c_int, [_P, C.POINTER(vc_solve_opts), C.POINTER(C.c_double), C.c_void_p,
                                 C.POINTER(vc_stats)]),
    "vc_capacitance_static": (C.c_int, [_P, C.POINTER(vc_solve_opts), C.POINTER(C.c_double), C.c_void_p,
                                        C.POINTER(vc_stats), _P]),
    "vc_capacitance_grad_eps": (C.c_int, [_P, C.POINTER(vc_solve_opts), C.POINTER(C.c_int32), C.c_int32,
                                          C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(vc_stats)]),
    "vc_update_eps": (C.c_int, [_P, C.POINTER(C.c_double), C.c_double, _P]),
    "vc_profile_enable": (C.c_int, [_P, C.c_int]),
    "vc_pass_times": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "vc_tuning_report": (C.c_int, [_P, C.c_char_p, C.c_int32]),
    "vc_capacitance_batch": (C.c_int, [C.POINTER(_P), C.c_int32, C.POINTER(vc_solve_opts), C.POINTER(C.c_void_p),
                                       C.POINTER(vc_stats)]),
    "vc_batch_capacitance": (C.c_int, [C.POINTER(_P), C.c_int32, C.POINTER(vc_solve_opts), C.POINTER(C.c_void_p),
                                       C.POINTER(vc_stats)]),
    "vc_pack_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.POINTER(_P)]),
    "vc_pack_destroy": (C.c_int, [_P]),
    "vc_pack_info": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "vc_pack_capacitance": (C.c_int, [_P, C.POINTER(vc_solve_opts), C.POINTER(C.c_void_p), C.POINTER(vc_stats)]),
    "vc_pack_apply": (C.c_int, [_P, C.c_int, C.c_void_p, C.c_void_p, _P]),
    "vc_tucker_info": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "vc_charges_to_capacitance": (C.c_int, [_P, _P, C.c_int32, _P, _P]),
    "vc_charges_to_capacitance_adjoint": (C.c_int, [_P, _P, C.c_int32, _P, _P]),
    "vc_xpass_candidates": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_int32), C.c_int32,
                                      C.POINTER(C.c_int32)]),
    "vc_xpass_set": (C.c_int, [_P, C.c_int, C.c_int, C.c_int32, C.POINTER(C.c_int32)]),
    "vc_ypass_set": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "vc_tuning_save": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_int32)]),
    "vc_tuning_load": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_int32)]),
    "vc_toeplitz_cache_build": (C.c_int, [C.POINTER(C.c_int32), C.c_double, C.c_int, _P, C.POINTER(_P)]),
    "vc_toeplitz_cache_destroy": (C.c_int, [_P]),
    "vc_toeplitz_cache_save": (C.c_int, [_P, C.c_char_p]),
    "vc_toeplitz_cache_load": (C.c_int, [C.c_char_p, C.c_int, C.POINTER(_P)]),
    "vc_toeplitz_cache_info": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "vc_toeplitz_cache_restore": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32), C.c_void_p, _P]),
    "vc_toeplitz_octant": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.c_int, C.c_void_p, _P]),
    "vc_setup_toeplitz_source": (C.c_int, [_P, _P]),
    "vc_setup_time": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "vc_memory_info": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "vc_status_string": (C.c_char_p, [C.c_int]),
    "vc_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
EXPORTED = tuple(_sig)


class VoxcapError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.vc_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.vc_status_string(status).decode()} ({status}): {msg}")


def _check(st, where, allow=()):
    if st != VC_OK and st not in allow:
        raise VoxcapError(st, where)
    return st


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return None
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ------------------------------------------------------------------ one-to-one wrappers
def vc_problem_create(cond_id, eps_r, dv, eps_background=1.0, device=0):
    cond_id = np.ascontiguousarray(cond_id, dtype=np.int32)
    eps_r = np.ascontiguousarray(eps_r, dtype=np.float64)
    if cond_id.ndim != 3 or cond_id.shape != eps_r.shape:
        raise ValueError("cond_id and eps_r must be equal 3-D arrays")
    g = vc_geometry(cond_id.shape[0], cond_id.shape[1], cond_id.shape[2], float(dv),
                    cond_id.ctypes.data_as(C.POINTER(C.c_int32)), eps_r.ctypes.data_as(C.POINTER(C.c_double)),
                    float(eps_background))
    h = _P()
    _check(_lib.vc_problem_create(C.byref(g), int(device), C.byref(h)), "vc_problem_create")
    return h


def vc_problem_destroy(h):
    return _lib.vc_problem_destroy(h)


def vc_panel_counts(h):
    nc, nd, m = C.c_int64(), C.c_int64(), C.c_int32()
    _check(_lib.vc_panel_counts(h, C.byref(nc), C.byref(nd), C.byref(m)), "vc_panel_counts")
    return nc.value, nd.value, m.value


def vc_panels(h):
    nc, nd, _ = vc_panel_counts(h)
    out = np.zeros(nc + nd, PANEL_DTYPE)
    _check(_lib.vc_panels(h, out.ctypes.data_as(C.c_void_p)), "vc_panels")
    return out


def vc_fft_size(h):
    m = (C.c_int32 * 3)()
    _check(_lib.vc_fft_size(h, m), "vc_fft_size")
    return tuple(m)


def vc_setup(h, fft_size=None, nv=None, tucker_tol=0.0, precisions=0, max_rhs=0, autotune=False, stream=None,
             tune_cache=None):
    o = vc_setup_opts()
    if fft_size is not None:
        o.fft_size[:] = [int(v) for v in fft_size]
    if nv is not None:
        o.nv[:] = [int(v) for v in (nv if np.ndim(nv) else (nv, nv, nv))]
    o.tucker_tol = float(tucker_tol)
    o.precisions = int(precisions)
    o.max_rhs = int(max_rhs)
    o.autotune = int(bool(autotune))
    o.tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
    _check(_lib.vc_setup(h, C.byref(o), _stream(stream)), "vc_setup")


def vc_apply(h, x, y, nrhs, transpose=False, prec="fp64", stream=None):
    _check(_lib.vc_apply(h, int(bool(transpose)), _PREC[prec], _ptr(x), _ptr(y), int(nrhs), _stream(stream)),
           "vc_apply")


def vc_apply_precond(h, x, y, nrhs, transpose=False, stream=None):
    _check(_lib.vc_apply_precond(h, int(bool(transpose)), _ptr(x), _ptr(y), int(nrhs), _stream(stream)),
           "vc_apply_precond")


def vc_apply_precond_kind(h, kind, x, y, nrhs, transpose=False, stream=None):
    _check(_lib.vc_apply_precond_kind(h, int(kind), int(bool(transpose)), _ptr(x), _ptr(y), int(nrhs),
                                      _stream(stream)), "vc_apply_precond_kind")


def vc_precond_info(h, kind):
    nbox, nblock, nbytes = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    _check(_lib.vc_precond_info(h, int(kind), C.byref(nbox), C.byref(nblock), C.byref(nbytes)), "vc_precond_info")
    return {"boxes": nbox.value, "distinct_blocks": nblock.value, "bytes": nbytes.value}


def vc_profile_enable(h, enable=True):
    """enable: False / 0 off, True / 1 events around every pass, 2 around the x pass only."""
    level = int(enable) if not isinstance(enable, bool) else int(enable)
    _check(_lib.vc_profile_enable(h, level), "vc_profile_enable")


PASS_NAMES = ("zfwd_scatter", "y_forward", "x_sandwich_multiply", "y_inverse", "zinv_gather")


def vc_charges_to_capacitance(h, rho, C_out, nrhs, stream=None):
    _check(_lib.vc_charges_to_capacitance(h, _ptr(rho), int(nrhs), _ptr(C_out), _stream(stream)),
           "vc_charges_to_capacitance")


def vc_charges_to_capacitance_adjoint(h, gC, grho, nrhs, stream=None):
    _check(_lib.vc_charges_to_capacitance_adjoint(h, _ptr(gC), int(nrhs), _ptr(grho), _stream(stream)),
           "vc_charges_to_capacitance_adjoint")


def vc_tucker_info(h):
    n = C.c_int32(0)
    ranks = (C.c_int32 * 45)()
    st, full, ms = C.c_double(0), C.c_double(0), C.c_double(0)
    cnt = C.c_int32(0)
    _check(_lib.vc_tucker_info(h, C.byref(n), ranks, C.byref(st), C.byref(full), C.byref(ms), C.byref(cnt)),
           "vc_tucker_info")
    r = [tuple(ranks[3 * q:3 * q + 3]) for q in range(n.value)]
    return {"npairs": n.value, "ranks": r, "stored_numbers": st.value, "full_numbers": full.value,
            "compression_ratio": (full.value / st.value) if st.value > 0 else None,
            "rebuild_ms": ms.value, "rebuilds": cnt.value}


def _n3(n):
    n = [int(v) for v in n]
    if len(n) != 3:
        raise ValueError("three sizes expected")
    return (C.c_int32 * 3)(*n)


def vc_toeplitz_cache_build(nmax, tol, device=0, stream=None):
    out = _P()
    _check(_lib.vc_toeplitz_cache_build(_n3(nmax), float(tol), int(device), _stream(stream), C.byref(out)),
           "vc_toeplitz_cache_build")
    return out


def vc_toeplitz_cache_destroy(h):
    _check(_lib.vc_toeplitz_cache_destroy(h), "vc_toeplitz_cache_destroy")


def vc_toeplitz_cache_save(h, path):
    _check(_lib.vc_toeplitz_cache_save(h, os.fsencode(path)), "vc_toeplitz_cache_save")


def vc_toeplitz_cache_load(path, device=0):
    out = _P()
    _check(_lib.vc_toeplitz_cache_load(os.fsencode(path), int(device), C.byref(out)), "vc_toeplitz_cache_load")
    return out


def vc_toeplitz_cache_info(h):
    nmax = (C.c_int32 * 3)()
    tol, stored, secs = C.c_double(0), C.c_double(0), C.c_double(0)
    ranks = (C.c_int32 * 45)()
    _check(_lib.vc_toeplitz_cache_info(h, nmax, C.byref(tol), ranks, C.byref(stored), C.byref(secs)),
           "vc_toeplitz_cache_info")
    nm = tuple(nmax)
    full = 15.0 * (nm[0] + 1) * (nm[1] + 1) * (nm[2] + 1)
    return {"nmax": nm, "tol": tol.value, "ranks": [tuple(ranks[3 * q:3 * q + 3]) for q in range(15)],
            "stored_numbers": stored.value, "full_numbers": full,
            "compression_ratio": full / stored.value if stored.value > 0 else None, "seconds": secs.value}


def vc_toeplitz_cache_restore(h, pair, n, out, stream=None):
    _check(_lib.vc_toeplitz_cache_restore(h, int(pair), _n3(n), _ptr(out), _stream(stream)),
           "vc_toeplitz_cache_restore")


def vc_toeplitz_octant(pair, n, out, device=0, stream=None):
    _check(_lib.vc_toeplitz_octant(int(pair), _n3(n), int(device), _ptr(out), _stream(stream)), "vc_toeplitz_octant")


def vc_setup_toeplitz_source(h, cache):
    _check(_lib.vc_setup_toeplitz_source(h, cache), "vc_setup_toeplitz_source")


def vc_setup_time(h):
    tot, tz = C.c_double(0), C.c_double(0)
    _check(_lib.vc_setup_time(h, C.byref(tot), C.byref(tz)), "vc_setup_time")
    return {"total_s": tot.value, "toeplitz_s": tz.value}


def vc_memory_info(h):
    sb, wb = C.c_double(0), C.c_double(0)
    _check(_lib.vc_memory_info(h, C.byref(sb), C.byref(wb)), "vc_memory_info")
    return {"spectra_bytes": sb.value, "work_bytes": wb.value}


def _octant_tensor(n, device):
    import torch
    n = [int(v) for v in n]
    return torch.empty((n[0] + 1, n[1] + 1, n[2] + 1), dtype=torch.float64, device=f"cuda:{device}")


def toeplitz_octant(pair, n, device=0):
    """Octant of Toeplitz pair `pair` for a grid of n voxels, from the panel integrals:
    a float64 CUDA tensor (n0+1, n1+1, n2+1)."""
    import torch
    out = _octant_tensor(n, device)
    vc_toeplitz_octant(pair, n, out, device, torch.cuda.current_stream(device))
    return out


class ToeplitzCache:
    """Owning wrapper of a vc_toeplitz_cache: the Tucker-compressed Toeplitz octants of
    every pair over a largest grid."""

    def __init__(self, handle, device):
        self._h = handle
        self.device = device

    @classmethod
    def build(cls, nmax, tol, device=0):
        import torch
        return cls(vc_toeplitz_cache_build(nmax, tol, device, torch.cuda.current_stream(device)), device)

    @classmethod
    def load(cls, path, device=0):
        return cls(vc_toeplitz_cache_load(path, device), device)

    def save(self, path):
        vc_toeplitz_cache_save(self._h, path)

    def info(self):
        return vc_toeplitz_cache_info(self._h)

    def restore(self, pair, n):
        """Restored octant of pair `pair` cropped to a grid of n voxels (float64 CUDA)."""
        import torch
        out = _octant_tensor(n, self.device)
        vc_toeplitz_cache_restore(self._h, pair, n, out, torch.cuda.current_stream(self.device))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            vc_toeplitz_cache_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _handles(handles):
    n = len(handles)
    return (_P * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])


def vc_pack_create(handles):
    out = _P()
    _check(_lib.vc_pack_create(_handles(handles), len(handles), C.byref(out)), "vc_pack_create")
    return out


def vc_pack_destroy(h):
    _check(_lib.vc_pack_destroy(h), "vc_pack_destroy")


def vc_pack_info(h):
    out = (C.c_int32 * 6)()
    _check(_lib.vc_pack_info(h, out), "vc_pack_info")
    keys = ("members", "columns", "rows", "launches_fp64", "launches_fp32", "launches_precond")
    return dict(zip(keys, (int(v) for v in out)))


def vc_pack_apply(h, x, y, prec="fp64", stream=None):
    """y = A x for every member at once; x, y: (columns, rows) float64 CUDA tensors."""
    _check(_lib.vc_pack_apply(h, _PREC[prec], _ptr(x), _ptr(y), _stream(stream)), "vc_pack_apply")


def vc_pack_capacitance(h, ms, allow_not_converged=False, **solve):
    o = _solve_opts(**solve)
    n = len(ms)
    Cs = [np.zeros((m, m)) for m in ms]
    outs = (C.c_void_p * n)(*[c.ctypes.data for c in Cs])
    st = (vc_stats * n)()
    status = _check(_lib.vc_pack_capacitance(h, C.byref(o), outs, st), "vc_pack_capacitance",
                    allow=(VC_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    return Cs, [stats_dict(st[k], ms[k]) for k in range(n)], status


def vc_capacitance_batch(handles, ms, allow_not_converged=False, **solve):
    """C matrices (list of m_k x m_k arrays) and stats of several set-up problems solved
    as one packed set (create, solve, free)."""
    o = _solve_opts(**solve)
    n = len(handles)
    hs = _handles(handles)
    Cs = [np.zeros((m, m)) for m in ms]
    outs = (C.c_void_p * n)(*[c.ctypes.data for c in Cs])
    st = (vc_stats * n)()
    status = _check(_lib.vc_capacitance_batch(hs, n, C.byref(o), outs, st), "vc_capacitance_batch",
                    allow=(VC_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    return Cs, [stats_dict(st[k], ms[k]) for k in range(n)], status


def vc_tuning_report(h):
    buf = C.create_string_buffer(8192)
    _check(_lib.vc_tuning_report(h, buf, len(buf)), "vc_tuning_report")
    return buf.value.decode()


def vc_tuning_save(h, path):
    n = C.c_int32(0)
    _check(_lib.vc_tuning_save(h, os.fsencode(path), C.byref(n)), "vc_tuning_save")
    return n.value


def vc_tuning_load(h, path):
    n = C.c_int32(0)
    _check(_lib.vc_tuning_load(h, os.fsencode(path), C.byref(n)), "vc_tuning_load")
    return n.value


def vc_xpass_candidates(h, prec="fp64", transpose=False):
    n = C.c_int32(0)
    _check(_lib.vc_xpass_candidates(h, _PREC[prec], int(bool(transpose)), None, 0, C.byref(n)),
           "vc_xpass_candidates")
    out = (C.c_int32 * (8 * max(1, n.value)))()
    _check(_lib.vc_xpass_candidates(h, _PREC[prec], int(bool(transpose)), out, n.value, C.byref(n)),
           "vc_xpass_candidates")
    rows = np.frombuffer(out, dtype=np.int32).reshape(-1, 8)[: n.value]
    return [tuple(int(v) for v in r) for r in rows]


def vc_xpass_set(h, cfg, prec="fp64", transpose=False, nrhs=1):
    arr = (C.c_int32 * 8)(*[int(v) for v in cfg])
    _check(_lib.vc_xpass_set(h, _PREC[prec], int(bool(transpose)), int(nrhs), arr), "vc_xpass_set")


def vc_ypass_set(h, kernel, cols=0, xcd_group=1, prec="fp64", transpose=False, inverse=False, nrhs=1):
    _check(_lib.vc_ypass_set(h, _PREC[prec], int(bool(transpose)), int(bool(inverse)), int(nrhs), int(kernel),
                             int(cols), int(xcd_group)), "vc_ypass_set")


def vc_pass_times(h):
    ms = (C.c_double * 5)()
    n = (C.c_int32 * 5)()
    b = (C.c_double * 5)()
    _check(_lib.vc_pass_times(h, ms, n, b), "vc_pass_times")
    return list(ms), list(n), list(b)


# VC_MIXED forms (vc_solve_opts.mixed_form)
_MIXED_FORM = {"auto": 0, "refinement": 1, "relaxed": 2}
MIXED_FORM_NAMES = {1: "refinement", 2: "relaxed"}


def _solve_opts(prec="fp64", rtol=0.0, restart=0, max_iter=0, inner_rtol=0.0, ir_max=0, use_precond=1, graph=True,
                mixed_form="auto"):
    o = vc_solve_opts()
    o.mixed_form = _MIXED_FORM[mixed_form]
    o.prec = _PREC[prec]
    o.rtol = rtol
    o.restart = restart
    o.max_iter = max_iter
    o.inner_rtol = inner_rtol
    o.ir_max = ir_max
    o.use_precond = use_precond
    o.graph = 0 if graph else 1
    return o


def vc_capacitance(h, m, rho=None, allow_not_converged=False, **solve):
    o = _solve_opts(**solve)
    Cm = np.zeros((m, m))
    st = vc_stats()
    status = _check(_lib.vc_capacitance(h, C.byref(o), Cm.ctypes.data_as(C.POINTER(C.c_double)), _ptr(rho),
                                        C.byref(st)), "vc_capacitance",
                    allow=(VC_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    return Cm, st, status


def vc_capacitance_static(h, m, rho=None, stream=None, **solve):
    o = _solve_opts(**solve)
    Cm = np.zeros((m, m))
    st = vc_stats()
    _check(_lib.vc_capacitance_static(h, C.byref(o), Cm.ctypes.data_as(C.POINTER(C.c_double)), _ptr(rho),
                                      C.byref(st), _stream(stream)), "vc_capacitance_static")
    return Cm, st


def vc_capacitance_grad_eps(h, m, block_of_voxel, nblocks, **solve):
    o = _solve_opts(**solve)
    blk = np.ascontiguousarray(block_of_voxel, dtype=np.int32)
    dC = np.zeros((nblocks, m, m))
    Cm = np.zeros((m, m))
    st = vc_stats()
    _check(_lib.vc_capacitance_grad_eps(h, C.byref(o), blk.ctypes.data_as(C.POINTER(C.c_int32)), int(nblocks),
                                        dC.ctypes.data_as(C.POINTER(C.c_double)),
                                        Cm.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st)),
           "vc_capacitance_grad_eps")
    return dC, Cm, st


def stats_dict(st, nrhs):
    return {"iters": list(st.iters[:nrhs]), "final_rre": list(st.final_rre[:nrhs]), "ir_steps": st.ir_steps,
            "mvp_count": st.mvp_count, "t_setup_s": st.t_setup_s, "t_solve_s": st.t_solve_s,
            "spectra_bytes": st.spectra_bytes, "bytes_model": st.bytes_model,
            "mixed_form": MIXED_FORM_NAMES.get(st.mixed_form), "steps_fp32": st.steps_fp32}


def capacitance_batch(problems, **solve):
    """Solve several set-up Problems together (uneven sizes welcome); returns
    ([C_k], [stats_k])."""
    Cs, sts, _ = vc_capacitance_batch([p._h for p in problems], [p.m for p in problems], **solve)
    return Cs, sts


def capacitance(cond_id, eps_r, dv, precision="fp64", eps_background=1.0, device=0, setup=None, **solve):
    """One-call form: (C, stats) of a voxel geometry (m x m farads, row-major), set up
    with the keyword options `setup` and solved with `solve` (rtol, restart, ...);
    precision "fp64", "mixed" or "fp32"."""
    P = Problem(cond_id, eps_r, dv, eps_background, device).setup(**dict(setup or {}))
    return P.capacitance(prec=precision, **solve)


class Pack:
    """Owning wrapper of a vc_pack: set-up Problems of any sizes solved as one (their
    products and preconditioner in shared launches).  Keeps the members alive; they
    must not be set up again while the pack exists."""

    def __init__(self, problems):
        self.members = list(problems)
        self._h = vc_pack_create([p._h for p in self.members])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            vc_pack_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return vc_pack_info(self._h)

    def apply(self, x, prec="fp64"):
        """Product of every member: x (columns, rows) float64 CUDA tensor -> y (same shape;
        rows past a member's panel count come back zero)."""
        import torch
        inf = self.info()
        if tuple(x.shape) != (inf["columns"], inf["rows"]) or x.dtype != torch.float64 or not x.is_cuda:
            raise ValueError(f"x must be a ({inf['columns']}, {inf['rows']}) float64 CUDA tensor")
        x = x.contiguous()
        y = torch.zeros_like(x)
        vc_pack_apply(self._h, x, y, prec=prec, stream=torch.cuda.current_stream())
        return y

    def capacitance(self, **solve):
        """([C_k], [stats_k]) for every member."""
        Cs, sts, _ = vc_pack_capacitance(self._h, [p.m for p in self.members], **solve)
        return Cs, sts


class Problem:
    """Owning wrapper of a vc_problem."""

    def __init__(self, cond_id, eps_r, dv, eps_background=1.0, device=0):
        self._h = vc_problem_create(cond_id, eps_r, dv, eps_background, device)
        self.n_cond, self.n_diel, self.m = vc_panel_counts(self._h)
        self.N = self.n_cond + self.n_diel
        self.device = device
        self.shape = tuple(int(v) for v in np.shape(cond_id))
        self.eps_background = float(eps_background)

    @classmethod
    def from_scene(cls, scene, device=0):
        return cls(scene["cond_id"], scene["eps_r"], scene["dv"], scene["eps_b"], device)

    def __del__(self):
        h = getattr(self, "_h", None)
        self._h = None
        # at interpreter exit the module's globals may already be gone: the process
        # releases the device memory then anyway
        if h and callable(vc_problem_destroy):
            try:
                vc_problem_destroy(h)
            except Exception:
                pass

    def panels(self):
        return vc_panels(self._h)

    def fft_size(self):
        return vc_fft_size(self._h)

    def setup(self, **kw):
        vc_setup(self._h, **kw)
        return self

    def set_toeplitz_source(self, cache):
        """Later setups take the Toeplitz tensors from `cache` (a ToeplitzCache), or from
        the panel integrals when None."""
        vc_setup_toeplitz_source(self._h, None if cache is None else cache._h)
        self._toeplitz_cache = cache   # kept alive for the setups that use it

    def spectra_bytes(self):
        """Device bytes held by the kernel spectra (stored, or the Tucker form)."""
        return vc_memory_info(self._h)["spectra_bytes"]

    def memory_info(self):
        return vc_memory_info(self._h)

    def setup_time(self):
        return vc_setup_time(self._h)

    def _vectors(self, x, y):
        """(x, y) checked for the C calls: (nrhs, N) contiguous float64 tensors on this
        problem's device (y allocated when None, distinct from x).  The library reads
        and writes nrhs * N doubles through the raw pointers, so anything else is
        refused here."""
        import torch

        def ok(t):
            return (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda and t.dim() == 2
                    and t.shape[1] == self.N and t.shape[0] >= 1
                    and (t.device.index if t.device.index is not None else torch.cuda.current_device()) == self.device)
        if not ok(x):
            raise ValueError(f"x must be a (nrhs, {self.N}) float64 tensor on cuda:{self.device}")
        x = x.contiguous()
        if y is None:
            return x, torch.empty_like(x)
        if not ok(y) or tuple(y.shape) != tuple(x.shape) or not y.is_contiguous():
            raise ValueError(f"y must be a contiguous float64 tensor of shape {tuple(x.shape)} on cuda:{self.device}")
        if y.data_ptr() == x.data_ptr():
            raise ValueError("y must not be x")
        return x, y

    def apply(self, x, y=None, transpose=False, prec="fp64", stream=None):
        """y = A x for x a (nrhs, N) float64 cuda tensor."""
        x, y = self._vectors(x, y)
        vc_apply(self._h, x, y, x.shape[0], transpose, prec, stream)
        return y

    def apply_precond(self, x, y=None, transpose=False, stream=None):
        x, y = self._vectors(x, y)
        vc_apply_precond(self._h, x, y, x.shape[0], transpose, stream)
        return y

    def apply_precond_kind(self, kind, x, y=None, transpose=False, stream=None):
        """y = R x for preconditioner kind 1 (eq. 14), 2 (diagonal) or 3 (block-diagonal
        over all panels, the comparison of Sec. III.A)."""
        x, y = self._vectors(x, y)
        vc_apply_precond_kind(self._h, kind, x, y, x.shape[0], transpose, stream)
        return y

    def precond_info(self, kind=1):
        """Boxes, distinct inverse blocks and stored bytes of preconditioner kind 1 or 3."""
        return vc_precond_info(self._h, kind)

    def profile(self, enable=True):
        vc_profile_enable(self._h, enable)

    def xpass_candidates(self, prec="fp64", transpose=False):
        """Rows (nst, r0..r5, cols) of the x-pass configurations this problem can use."""
        return vc_xpass_candidates(self._h, prec, transpose)

    def xpass_set(self, cfg, prec="fp64", transpose=False, nrhs=1):
        vc_xpass_set(self._h, cfg, prec, transpose, nrhs)

    def ypass_set(self, kernel, cols=0, xcd_group=1, prec="fp64", transpose=False, inverse=False, nrhs=1):
        vc_ypass_set(self._h, kernel, cols, xcd_group, prec, transpose, inverse, nrhs)

    def tucker_info(self):
        """Ranks, compression ratio and rebuild timing of the Tucker-compressed spectra."""
        return vc_tucker_info(self._h)

    def tuning_report(self):
        """Launch configurations of the x and y passes in use (and what the autotuner measured)."""
        return vc_tuning_report(self._h)

    def save_tuning(self, path):
        """Merge the timed x- and y-pass choices into the cache file `path`; returns how many."""
        return vc_tuning_save(self._h, path)

    def load_tuning(self, path):
        """Adopt the cached x- and y-pass choices of `path` that fit this problem; returns how many."""
        return vc_tuning_load(self._h, path)

    def pass_times(self):
        """(ms summed, launches, algorithmic bytes of one launch) per pass of the product."""
        return vc_pass_times(self._h)

    def capacitance(self, rho=None, **solve):
        Cm, st, _ = vc_capacitance(self._h, self.m, rho=rho, **solve)
        return Cm, stats_dict(st, self.m)

    def capacitance_static(self, rho=None, stream=None, **solve):
        """capacitance() with the solve's device arrays in the library's static scratch
        (vc_capacitance_static: no device allocation, no graphs)."""
        if rho is not None:
            rho_c, _ = self._vectors(rho, None)
            if rho_c.shape[0] != self.m or rho_c.data_ptr() != rho.data_ptr():
                raise ValueError(f"rho must be a contiguous ({self.m}, {self.N}) float64 tensor on cuda:{self.device}")
        Cm, st = vc_capacitance_static(self._h, self.m, rho=rho, stream=stream, **solve)
        return Cm, stats_dict(st, self.m)

    def update_eps(self, eps_r, eps_background=None, stream=None):
        """New non-conductor permittivities (grid-shaped) without a new setup; the panel
        list must stay the same (else VoxcapError with status VC_ERR_ARG)."""
        e = np.ascontiguousarray(eps_r, dtype=np.float64)
        if e.shape != self.shape:
            raise ValueError(f"eps_r must have the grid's shape {self.shape}")
        eb = self.eps_background if eps_background is None else float(eps_background)
        _check(_lib.vc_update_eps(self._h, e.ctypes.data_as(C.POINTER(C.c_double)), eb, _stream(stream)),
               "vc_update_eps")
        self.eps_background = eb
        return self

    def capacitance_grad_eps(self, block_of_voxel, nblocks, **solve):
        dC, Cm, st = vc_capacitance_grad_eps(self._h, self.m, block_of_voxel, nblocks, **solve)
        return dC, Cm, stats_dict(st, self.m)
