"""Test-side glue between the library's panel order / row convention and the oracle's."""
import numpy as np

import oracle


def library_panels_to_oracle(lib_panels, po):
    """perm such that oracle index perm[i] is the library panel i."""
    key_o = {}
    for t in range(len(po["axis"])):
        key_o[(int(po["axis"][t]), int(po["idx"][t, 0]), int(po["idx"][t, 1]), int(po["idx"][t, 2]))] = t
    perm = np.array([key_o[(int(p["dir"]), int(p["i"]), int(p["j"]), int(p["k"]))] for p in lib_panels])
    return perm


def oracle_matrix_library_order(scene, lib_panels):
    """Dense eq. (4) matrix in library order with dielectric rows written for the +axis
    normal (the paper's row times its orientation sign), as the library applies it."""
    po = oracle.panelize(scene["cond_id"], scene["eps_r"], scene["eps_b"])
    A = oracle.assemble(po)
    S = np.where(po["kind"] == 1, po["sign"], 1).astype(float)
    A = S[:, None] * A
    perm = library_panels_to_oracle(lib_panels, po)
    return A[np.ix_(perm, perm)], po, perm
