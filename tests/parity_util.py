"""Relative errors of slab-major space-time vectors, whole and per variable block.

The blocks u (both velocity components), p, j and A differ in scale by orders
of magnitude, so a parity check asserts the relative error of each block over
all slabs as well as that of the whole vector: an error confined to a small
block cannot hide under the whole-vector norm.
"""
import numpy as np

BLOCKS = ("u", "p", "j", "A")


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def block_errors(a, b, offsets, nt):
    """{'all', 'u', 'p', 'j', 'A'} -> relative 2-norm error of a against b.
    offsets = [u_x, u_y, p, j, A, end] within one slab of the slab-major layout."""
    ns = offsets[5]
    A = np.asarray(a).reshape(nt, ns)
    B = np.asarray(b).reshape(nt, ns)
    cuts = {"u": (offsets[0], offsets[2]), "p": (offsets[2], offsets[3]), "j": (offsets[3], offsets[4]),
            "A": (offsets[4], offsets[5])}
    out = {"all": rel(A, B)}
    for name, (lo, hi) in cuts.items():
        if hi > lo:
            out[name] = rel(A[:, lo:hi], B[:, lo:hi])
    return out


def assert_blocks(a, b, offsets, nt, tol, what=""):
    e = block_errors(a, b, offsets, nt)
    print(f"    {what} " + " ".join(f"{k}={v:.1e}" for k, v in e.items()), flush=True)
    bad = {k: v for k, v in e.items() if not v <= tol}
    assert not bad, (what, bad, tol)
    return e
