"""Helpers shared by the GPU tests (comparison against the oracle)."""
import numpy as np


def rel_err_per_l(z, ref):
    """max_{b1,b2} |z_l - ref_l| / max_{b1,b2} |ref_l| for every l (global max when ref_l = 0)."""
    glob = np.abs(ref).max()
    out = []
    for l in range(ref.shape[0]):
        scale = np.abs(ref[l]).max()
        if scale == 0.0:
            scale = glob if glob > 0 else 1.0
        out.append(np.abs(z[l] - ref[l]).max() / scale)
    return np.array(out)


def say(*a):
    print(*a, flush=True)
