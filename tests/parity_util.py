"""Helpers shared by the GPU parity tests: run the same seeded case through the
HIP library (via its Python binding) and through the FP64 oracle, and compare
macroscopic fields with the error definitions used throughout the suite."""
import numpy as np

from oracle.oracle import Oracle, OracleParams


def gpu_case(shape, solid, xi, rho, tau, G, g, storage=0):
    import torch
    from paper_2207_01534_amd.lattice import Lattice, LatticeParams, Storage
    p = LatticeParams(shape=shape, tau=tau, G=G, g=g, storage=Storage(storage))
    lat = Lattice(p, torch.as_tensor(solid), torch.as_tensor(np.asarray(xi, np.float32)),
                  torch.as_tensor(np.asarray(rho, np.float32)))
    return lat


def oracle_case(shape, solid, xi, rho, tau, G, g):
    """The oracle is fed exactly the float32 inputs the GPU sees, widened to FP64."""
    o = Oracle(OracleParams(shape, tau=tau, G=G, g=g), solid,
               np.asarray(xi, np.float32).astype(np.float64))
    rho32 = np.asarray(rho, np.float32).astype(np.float64)
    rho32[:, solid != 0] = 0.0
    o.init_equilibrium(rho32)
    return o


def gpu_fields(lat):
    import torch
    torch.cuda.synchronize()
    r = lat.density().cpu().numpy().astype(np.float64)
    u = lat.velocity().cpu().numpy().astype(np.float64)
    F = lat.force().cpu().numpy().astype(np.float64)
    P = lat.pressure().cpu().numpy().astype(np.float64)
    return r, u, F, P


def field_errors(gpu, orc, solid):
    """e_rho (per component, normalised by the field max), e_u, e_F, per-node relative rho error."""
    r, u, F, P = gpu
    ro, uo, Fo, Po = orc
    fl = solid == 0
    e_rho = max(np.abs(r[s][fl] - ro[s][fl]).max() / np.abs(ro[s][fl]).max() for s in range(2))
    rel_node = max((np.abs(r[s][fl] - ro[s][fl]) / np.abs(ro[s][fl])).max() for s in range(2))
    un = np.sqrt((uo ** 2).sum(0))[fl].max()
    e_u = np.sqrt(((u - uo) ** 2).sum(0))[fl].max() / max(un, 1e-30)
    Fn = np.abs(Fo).max()
    e_F = np.abs(F - Fo).max() / max(Fn, 1e-30)
    e_P = np.abs(P - Po)[fl].max() / np.abs(Po[fl]).max()
    return dict(e_rho=e_rho, rel_node=rel_node, e_u=e_u, e_F=e_F, e_P=e_P, u_max=un)


def oracle_fields(o):
    r, _, F, u = o.fields()
    P = o.pressure()
    return r, u, F, P
