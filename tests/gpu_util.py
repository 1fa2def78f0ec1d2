"""Helpers for the GPU parity tests: move seeded inputs and states between the
oracle's numpy arrays and the library (direction order mapped through the
velocity tables, never assumed)."""
import numpy as np

from oracle.lattice import E19, E7


def dir_perm(gpu_e, oracle_e):
    """p with gpu direction i == oracle direction p[i]."""
    idx = {tuple(v): a for a, v in enumerate(oracle_e)}
    return np.array([idx[tuple(v)] for v in gpu_e])


def perms():
    import paper_0809_4730_amd as pkg
    p19 = dir_perm(pkg.lattice_velocities(19), E19)
    p7 = dir_perm(pkg.lattice_velocities(7), E7)
    return p19, p7


def to_gpu_f(d, torch_dtype, device="cuda"):
    import torch
    p19, _ = perms()
    return torch.tensor(np.ascontiguousarray(d[p19]), dtype=torch.float64, device=device).to(torch_dtype)


def from_gpu_f(t):
    import torch
    p19, _ = perms()
    arr = t.to(torch.float64).cpu().numpy()
    out = np.empty_like(arr)
    out[p19] = arr
    return out


def _rest_g(g_shape, B0):
    from oracle.lattice import W7
    rest = np.zeros(g_shape)
    for j in range(3):
        for a in range(7):
            rest[j, a] = W7[a] * B0[j]
    return rest


def to_gpu_g(g, torch_dtype, B0, device="cuda"):
    """Oracle magnetic populations -> library state (deviations from W B0)."""
    import torch
    _, p7 = perms()
    dev = g - _rest_g(g.shape, B0)
    return torch.tensor(np.ascontiguousarray(dev[:, p7]), dtype=torch.float64, device=device).to(torch_dtype)


def from_gpu_g(t, B0):
    _, p7 = perms()
    arr = t.to(__import__("torch").float64).cpu().numpy()
    out = np.empty_like(arr)
    out[:, p7] = arr
    return out + _rest_g(out.shape, B0)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def announce(msg):
    print(msg, flush=True)
