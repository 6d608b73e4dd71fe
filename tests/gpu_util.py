"""Helpers shared by the GPU parity tests: device transfer, comparison metrics,
and mapping the library's cell-ordered ion arrays back to ids."""
import numpy as np

TOL = 1e-10  # relative L2 bar for fields, forces, velocities and displacements


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    num = np.linalg.norm((a - b).ravel())
    return num / den if den > 0 else num


def dev(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a.copy())
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def min_image(d, L):
    d = np.array(d, dtype=np.float64)
    for k in range(2):
        d[k] -= L[k] * np.round(d[k] / L[k])
    return d


def by_id(pos, ids, want):
    """Columns of pos for the ion ids `want` (ids are a permutation of 0..n-1)."""
    where = np.empty(len(ids), dtype=np.int64)
    where[ids] = np.arange(len(ids))
    return pos[:, where[want]]


def log(msg):
    print(msg, flush=True)
