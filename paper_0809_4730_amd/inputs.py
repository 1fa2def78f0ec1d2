"""Seeded synthetic inputs shared by the tests, the bench and the oracle runs.

Only input construction lives here (force fields, random population
deviations, physical-parameter conversions of the workloads); none of the
method's arithmetic.  Everything is numpy, deterministic for a given seed.

Workloads (lattice units, nodes at k + 1/2 between walls at 0 and n):

* plane Poiseuille: uniform F = (F, 0, 0), walls normal to z (Sec. 5);
* square duct: F_x = F0 sin(2 pi y / ny) (1 + cos(2 pi z / nz) / 2), walls
  normal to y and z, periodic x;
* Hartmann: uniform F_x, applied field B0 along y (the wall normal),
  Ha = B0 L / sqrt(mu eta rho nu) with half-width L = ny / 2, and the chi
  scaling Pm_eff = chi nu / eta (Sec. 4.1, Sec. 5).
"""
import numpy as np


def duct_force(shape, F0=1e-5, dtype=np.float64):
    """(3, nz, ny, nx) force of the square-duct workload."""
    nx, ny, nz = shape
    y = np.arange(ny) + 0.5
    z = np.arange(nz) + 0.5
    F = np.zeros((3, nz, ny, nx), dtype=dtype)
    F[0] = (F0 * np.sin(2 * np.pi * y / ny)[None, :, None]
            * (1.0 + 0.5 * np.cos(2 * np.pi * z / nz))[:, None, None])
    return F


def uniform_force(shape, F, dtype=np.float64):
    nx, ny, nz = shape
    out = np.empty((3, nz, ny, nx), dtype=dtype)
    for a in range(3):
        out[a] = F[a]
    return out


def random_deviations(shape, seed, amp=1e-4, q=19, dtype=np.float64):
    """Population deviations amp * U(-1, 1), shape (q, nz, ny, nx)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return (amp * rng.uniform(-1.0, 1.0, (q, nz, ny, nx))).astype(dtype)


def random_force(shape, seed, amp=1e-5, dtype=np.float64):
    nx, ny, nz = shape
    rng = np.random.default_rng(10_000 + seed)
    return (amp * rng.uniform(-1.0, 1.0, (3, nz, ny, nx))).astype(dtype)


def random_nodes(shape, count, seed):
    """count distinct (x, y, z) nodes, always including the eight corners."""
    nx, ny, nz = shape
    rng = np.random.default_rng(20_000 + seed)
    corners = np.array([(x, y, z) for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)])
    N = nx * ny * nz
    idx = rng.choice(N, size=min(count, N), replace=False)
    pts = np.stack([idx % nx, (idx // nx) % ny, idx // (nx * ny)], axis=1)
    return np.unique(np.concatenate([corners, pts]), axis=0)


def hartmann_parameters(Ha, Pm, ny, nu=0.1, eta=0.025, rho=1.0, mu=1.0):
    """(B0, chi) for Hartmann number Ha and effective magnetic Prandtl number Pm
    on a channel of ny nodes between walls normal to y."""
    L = ny / 2.0
    B0 = Ha * np.sqrt(mu * eta * rho * nu) / L
    chi = Pm * eta / nu
    return B0, chi


def cavity_field(Ha, Pm, W, nu, eta, rho=1.0, mu=1.0):
    """(B0, chi) for Hartmann number Ha = B0 W / sqrt(mu eta rho nu) on a cavity
    of side W and effective magnetic Prandtl number Pm = chi nu / eta."""
    return Ha * np.sqrt(mu * eta * rho * nu) / W, Pm * eta / nu


# Workload presets (sizes and parameters of the configurations measured).
POISEUILLE = dict(shape=(8, 8, 32), bc=("periodic", "periodic", "wall"), F=(1e-6, 0.0, 0.0),
                  nu=0.1, gammas=(1.0, 0.1), tol=1e-10)
DUCT64 = dict(shape=(64, 64, 64), bc=("periodic", "wall", "wall"), F0=1e-5, nu=0.131,
              gammas=(1.0, 0.5, 0.1, 0.05), tol=1e-8)
HARTMANN = dict(shape=(32, 32, 128), bc=("periodic", "wall", "periodic"), F=(1e-5, 0.0, 0.0),
                nu=0.1, eta=0.025, gamma=0.1, gamma_m=0.1, Ha=(5.0, 10.0, 20.0), Pm=(0.01, 0.1),
                tol=1e-8)
DUCT256 = dict(shape=(256, 256, 256), bc=("periodic", "wall", "wall"), F0=1e-5, nu=0.131,
               gamma=1.0)
ADJOINT = dict(shape=(128, 128, 128), bc=("periodic", "wall", "wall"), F0=1e-5, nu=0.131,
               gamma=1.0, unrolled_shape=(32, 32, 32), unrolled_steps=2000, ckpt_every=45)
MHD_CAVITY = dict(W=64, U0=0.0235, nu=0.015, eta=0.015, Ha=45.0, Pm=5.625e-7, pad=16,
                  gammas=(1.0, 0.5, 0.1), tol=1e-6)
