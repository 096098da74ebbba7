"""Seeded synthetic inputs for the two-component LBM step.

This module builds geometry and initial-condition arrays only; it holds none
of the lattice Boltzmann arithmetic, so both the HIP library's callers and the
FP64 test oracle may consume it.  Everything is NumPy, deterministic for a
given seed, and returns C-ordered arrays of shape (nz, ny, nx) (x fastest).

Stand-ins for the paper's data (Sec. 4): the Finney sphere pack and the
Bentheimer micro-CT volume are not available, so sphere packs and thresholded
Gaussian random fields of the same kind are generated here.

Conventions: component 1 is the non-wetting invader ("oil"), component 2 the
wetting phase ("water"); majority density 1.0, minority 0.03.
"""
from dataclasses import dataclass, field
import hashlib

import numpy as np

RHO_MAJOR = 1.0
RHO_MINOR = 0.03


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def tanh_droplet(shape, radius, center=None, rho_in=RHO_MAJOR, rho_out=RHO_MINOR, width=5.0):
    """Diffuse-interface droplet of component 1 in component 2 (Sec. 3.1, Eq. 16).

    Returns rho of shape (2, nz, ny, nx).  The centre defaults to the domain
    centre ((n-1)/2 on each axis) so that the lattice reflections map the
    initial field onto itself.
    """
    nx, ny, nz = shape
    if center is None:
        center = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    t = np.tanh(2.0 * (r - radius) / width)
    rho1 = 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * t
    rho2 = 0.5 * (rho_in + rho_out) + 0.5 * (rho_in - rho_out) * t
    return np.stack([rho1, rho2])


def sphere_pack(shape, radius, porosity, seed, buffer=3, overlap=True, max_spheres=10_000_000):
    """Solid mask of randomly placed spheres, periodic in y and z.

    Sphere centres are drawn uniformly in the sample region x in
    [buffer, nx-buffer) and added one at a time until the sample porosity
    falls to ``porosity`` or below.  With ``overlap=True`` spheres may overlap
    (Boolean model); hard-sphere random sequential addition jams near a solid
    fraction of 0.38 and cannot reach porosity 0.40.  Voxel (x, y, z) is solid
    iff its integer centre lies within ``radius`` of a sphere centre (periodic
    images in y and z).  The buffers stay fluid.

    Returns (mask uint8 (nz, ny, nx), info dict).
    """
    nx, ny, nz = shape
    rng = _rng(seed)
    solid = np.zeros((nz, ny, nx), np.uint8)
    x0, x1 = buffer, nx - buffer
    sample_vol = (x1 - x0) * ny * nz
    n_solid = 0
    R = int(np.ceil(radius))
    off = np.arange(-R, R + 1)
    dz, dy, dx = np.meshgrid(off, off, off, indexing="ij")
    ball = (dx ** 2 + dy ** 2 + dz ** 2) <= radius * radius
    bdz, bdy, bdx = dz[ball], dy[ball], dx[ball]
    centres = []
    n_tries = 0
    while 1.0 - n_solid / sample_vol > porosity and len(centres) < max_spheres:
        n_tries += 1
        c = (rng.uniform(x0, x1), rng.uniform(0, ny), rng.uniform(0, nz))
        ci = np.floor(np.array(c)).astype(np.int64)
        xs = ci[0] + bdx
        ys = (ci[1] + bdy) % ny
        zs = (ci[2] + bdz) % nz
        keep = (xs >= x0) & (xs < x1)
        xs, ys, zs = xs[keep], ys[keep], zs[keep]
        if not overlap and solid[zs, ys, xs].any():
            if n_tries > 200 * (len(centres) + 100):
                break
            continue
        newly = solid[zs, ys, xs] == 0
        n_solid += int(newly.sum())
        solid[zs, ys, xs] = 1
        centres.append(c)
    info = {"spheres": len(centres), "porosity": 1.0 - n_solid / sample_vol,
            "porosity_total": 1.0 - solid.mean()}
    return solid, info


def gaussian_field_medium(shape, ell, porosity, seed, buffer=3):
    """Thresholded Gaussian random field (sandstone-like stand-in).

    White noise N(0,1) is filtered periodically with a Gaussian kernel so
    that the field covariance is exp(-r^2 / (2 ell^2)); a voxel of the sample
    region is pore iff its value is at or below the ``porosity`` quantile.
    Isolated pores are kept.  Buffers of ``buffer`` planes at both x ends stay
    fluid.  Returns (mask uint8 (nz, ny, nx), info dict).
    """
    nx, ny, nz = shape
    rng = _rng(seed)
    noise = rng.standard_normal((nz, ny, nx))
    # Kernel std sigma = ell / sqrt(2) gives covariance std ell.
    sigma = ell / np.sqrt(2.0)
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    filt = np.exp(-2.0 * (np.pi * sigma) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    fieldv = np.fft.irfftn(np.fft.rfftn(noise) * filt, s=(nz, ny, nx), axes=(0, 1, 2))
    sample = fieldv[:, :, buffer:nx - buffer]
    thr = np.quantile(sample, porosity)
    solid = (fieldv > thr).astype(np.uint8)
    solid[:, :, :buffer] = 0
    solid[:, :, nx - buffer:] = 0
    info = {"porosity": 1.0 - solid[:, :, buffer:nx - buffer].mean(),
            "porosity_total": 1.0 - solid.mean()}
    return solid, info


def _clusters(mask):
    """Cluster ids of a boolean mask (nz, ny, nx): voxels are connected when
    they are D3Q19 neighbours (sharing a face or an edge), periodically in y
    and z, not in x.  Returns an int array, 0 outside the mask."""
    from scipy import ndimage
    m = np.pad(mask, ((1, 1), (1, 1), (0, 0)), mode="wrap")          # one periodic copy layer in z, y
    lab, n = ndimage.label(m, structure=ndimage.generate_binary_structure(3, 2))
    parent = np.arange(n + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    # a copy-layer voxel is the same voxel as its periodic original: join their clusters
    core = lab[1:-1, 1:-1, :]
    pairs = [(lab[0, 1:-1, :], core[-1]), (lab[-1, 1:-1, :], core[0]),
             (lab[1:-1, 0, :], core[:, -1]), (lab[1:-1, -1, :], core[:, 0])]
    zy = [(0, 0, -1, -1), (0, -1, -1, 0), (-1, 0, 0, -1), (-1, -1, 0, 0)]   # the four copied edges
    pairs += [(lab[a, b, :], core[c, d]) for a, b, c, d in zy]
    for u, v in pairs:
        both = (u > 0) & (v > 0)
        for a, b in np.unique(np.stack([u[both], v[both]], axis=1), axis=0):
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[ra] = rb
    roots = np.array([find(a) for a in range(n + 1)])
    return roots[core]


def percolating_fraction(solid, buffer=3):
    """Fraction of the sample's pore voxels (x in [buffer, nx - buffer)) that
    belong to a pore cluster joining the inlet buffer (x < buffer) to the
    outlet buffer (x >= nx - buffer) through the sample (clusters as in
    _clusters)."""
    nx = solid.shape[2]
    pore = solid == 0
    root = _clusters(pore)
    inlet = np.unique(root[:, :, :buffer][pore[:, :, :buffer]])
    outlet = np.unique(root[:, :, nx - buffer:][pore[:, :, nx - buffer:]])
    spanning = np.intersect1d(inlet, outlet)
    sample = pore[:, :, buffer:nx - buffer]
    if not sample.any():
        return 0.0
    return float(np.isin(root[:, :, buffer:nx - buffer][sample], spanning).mean())


def trapped_region(rho, solid, buffer=3):
    """Trapped non-wetting phase: fluid voxels where component 1 dominates
    (rho1 > rho2) that belong to a component-1 cluster (as in _clusters) not
    reaching the inlet buffer (x < buffer).  Returns a uint8 mask, the frozen
    region of the trapped-saturation loss."""
    nw = (solid == 0) & (np.asarray(rho[0]) > np.asarray(rho[1]))
    root = _clusters(nw)
    inlet = np.unique(root[:, :, :buffer][nw[:, :, :buffer]])
    return (nw & ~np.isin(root, inlet)).astype(np.uint8)


def ganglia_rho(solid, n_blobs, radius, seed, buffer=3, width=2.5):
    """Component 1 (non-wetting) as dispersed blobs of the given radius centred
    at seeded random pore voxels, plus the inlet buffer; component 2 elsewhere.
    Each blob and the reservoir carry a tanh interface of the given width;
    densities RHO_MAJOR / RHO_MINOR, 0 at solid voxels."""
    nz, ny, nx = solid.shape
    rng = _rng(seed)
    pores = np.argwhere(solid[:, :, buffer + int(radius):nx - buffer - int(radius)] == 0)
    pick = pores[rng.choice(len(pores), size=n_blobs, replace=False)]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = 0.5 * (1.0 + np.tanh(2.0 * (buffer - 0.5 - x) / width))          # inlet reservoir
    for cz, cy, cx in pick:
        cx = cx + buffer + int(radius)
        dz = (z - cz + nz / 2.0) % nz - nz / 2.0
        dy = (y - cy + ny / 2.0) % ny - ny / 2.0
        d = np.sqrt((x - cx) ** 2 + dy ** 2 + dz ** 2)
        phi = np.maximum(phi, 0.5 * (1.0 - np.tanh(2.0 * (d - radius) / width)))
    r1 = RHO_MINOR + (RHO_MAJOR - RHO_MINOR) * phi
    r2 = RHO_MINOR + (RHO_MAJOR - RHO_MINOR) * (1.0 - phi)
    rho = np.stack([r1, r2])
    rho[:, solid != 0] = 0.0
    return rho


def uniform_xi(solid, lo, hi, seed):
    """Per-voxel adhesion parameter, i.i.d. U[lo, hi] at solid voxels, 0 elsewhere (float32)."""
    rng = _rng(seed)
    xi = rng.uniform(lo, hi, size=solid.shape).astype(np.float32)
    xi[solid == 0] = 0.0
    return xi


def constant_xi(solid, value):
    xi = np.zeros(solid.shape, np.float32)
    xi[solid != 0] = np.float32(value)
    return xi


def inlet_drainage_rho(solid, buffer=3, width=5.0):
    """Component 1 fills the fluid reservoir formed by the inlet buffer (x < buffer)
    and, across the periodic x boundary, the outlet buffer (x >= nx - buffer);
    component 2 fills the rest.  The two interfaces carry the diffuse tanh
    profile of the paper's initialisation (Sec. 3.1, Eq. 16) in one dimension,
    with width W = 5, centred on the buffer edges."""
    nz, ny, nx = solid.shape
    x = np.arange(nx, dtype=np.float64)
    centre = -0.5                              # between x = nx - 1 and x = 0
    d = np.abs((x - centre + nx / 2.0) % nx - nx / 2.0)   # periodic distance to the centre
    half = float(buffer)                       # reservoir spans both buffers
    t = np.tanh(2.0 * (d - half) / width)
    r1 = 0.5 * (RHO_MAJOR + RHO_MINOR) - 0.5 * (RHO_MAJOR - RHO_MINOR) * t
    r2 = (RHO_MAJOR + RHO_MINOR) - r1
    rho = np.stack([np.broadcast_to(r1, (nz, ny, nx)), np.broadcast_to(r2, (nz, ny, nx))]).copy()
    rho[:, solid != 0] = 0.0
    return rho


def open_drainage_rho(solid, front=6.0, width=5.0):
    """Initial densities for a drainage driven through open x planes: component 1
    fills the inlet side up to a front at x = front (inside the fluid buffer
    layers and the first pore layer), component 2 the rest, outlet buffer
    included, with the diffuse tanh interface of the paper's initialisation
    (Sec. 3.1, Eq. 16) in one dimension, width W = 5.  Unlike
    inlet_drainage_rho the outlet holds the displaced component, as the
    outlet condition (component 2 imposed) requires."""
    nz, ny, nx = solid.shape
    x = np.arange(nx, dtype=np.float64)
    t = np.tanh(2.0 * (x - front) / width)
    r1 = 0.5 * (RHO_MAJOR + RHO_MINOR) - 0.5 * (RHO_MAJOR - RHO_MINOR) * t
    r2 = (RHO_MAJOR + RHO_MINOR) - r1
    rho = np.stack([np.broadcast_to(r1, (nz, ny, nx)), np.broadcast_to(r2, (nz, ny, nx))]).copy()
    rho[:, solid != 0] = 0.0
    return rho


def open_drainage(w: "Workload", reservoir: int = 10) -> "Workload":
    """The workload's sample set up for a drainage driven through open x planes:
    the first and last `reservoir` x planes are cleared of solid (pure-fluid
    inlet and outlet reservoirs, as the paper adds in front of and behind its
    samples, Sec. 4.1), component 1 fills the inlet reservoir up to two planes
    short of the sample (open_drainage_rho), and the body force is zero (the
    imposed inlet/outlet densities drive the flow)."""
    solid = w.solid.copy()
    solid[:, :, :reservoir] = 0
    solid[:, :, solid.shape[2] - reservoir:] = 0
    xi = np.where(solid != 0, w.xi, 0).astype(np.float32)
    rho = open_drainage_rho(solid, front=reservoir - 2.0)
    info = dict(w.info, reservoir=reservoir)
    return Workload(w.name + "+open", w.shape, solid, xi, rho, w.tau, w.G, ((0, 0, 0), (0, 0, 0)), w.steps, info)


def contact_angle_cubic(xi):
    """The paper's fitted contact angle (degrees) versus xi (Sec. 3.2)."""
    return 47.4136 * xi ** 3 - 23.4513 * xi ** 2 + 89.7938 * xi + 91.2324


# Adhesion parameter for a 45 degree contact angle through component 2 at the
# porous workloads' viscosity ratio M = 10 (tau = 1.5, 0.6), G = 3.5,
# densities 1 / 0.027: the oracle's flat-wall half drop (quasi-2D, 120 x 60,
# R0 = 22, 8000 steps) gives 45.33 degrees at xi = -0.470 and 44.72 at -0.475,
# interpolated here; the root of the paper's Sec. 3.2 cubic, -0.426, gives
# 50.4 degrees on the same drop.
XI45_M10 = -0.473


def xi_for_angle(theta_deg):
    """Real root in [-1, 1] of the paper's cubic for a target contact angle."""
    roots = np.roots([47.4136, -23.4513, 89.7938, 91.2324 - theta_deg])
    real = [r.real for r in roots if abs(r.imag) < 1e-9 and -1.0 <= r.real <= 1.0]
    return float(real[0])


def random_state(shape, seed, lo=0.5, hi=1.5):
    """Random positive populations (2, 19, nz, ny, nx) for unit tests (float64)."""
    nx, ny, nz = shape
    rng = _rng(seed)
    return rng.uniform(lo, hi, size=(2, 19, nz, ny, nx)) / 19.0


def random_mask(shape, fraction, seed):
    nx, ny, nz = shape
    rng = _rng(seed)
    return (rng.uniform(size=(nz, ny, nx)) < fraction).astype(np.uint8)


def sha256(arr) -> str:
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()


@dataclass
class Workload:
    name: str
    shape: tuple
    solid: np.ndarray
    xi: np.ndarray            # float32 (nz, ny, nx)
    rho: np.ndarray           # float64 (2, nz, ny, nx) initial densities
    tau: tuple
    G: float
    g: tuple
    steps: int
    info: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return int(np.prod(self.shape))

    @property
    def n_fluid(self):
        return int((self.solid == 0).sum())


def workload(name: str, shape=None) -> Workload:
    """The five standard workloads (optionally at a reduced shape for tests).

    droplet32     32^3 periodic droplet, r = 8, G = 0.9, tau = (1, 1), 200 steps
    spheres128    128^3 overlapping-sphere pack r = 8, porosity 0.40, seed 2207,
                  M = 10 (tau 1.5 / 0.6), xi for 45 degrees at M = 10 (XI45_M10),
                  g1 = 5e-4 x-hat
    gauss256      256^3 Gaussian field ell = 4, porosity 0.22, seed 1534, M = 10
    spheres512    512^3 sphere pack r = 12, porosity 0.38, seed 512, M = 10
    adjoint64     64^3 sphere pack r = 6, porosity 0.40, seed 64, xi ~ U[-0.4, 0.4]
    """
    xi45 = XI45_M10
    if name == "droplet32":
        shape = shape or (32, 32, 32)
        nx, ny, nz = shape
        solid = np.zeros((nz, ny, nx), np.uint8)
        rho = tanh_droplet(shape, radius=8.0 * nx / 32.0)
        return Workload(name, shape, solid, np.zeros(solid.shape, np.float32), rho,
                        (1.0, 1.0), 0.9, ((0, 0, 0), (0, 0, 0)), 200)
    g_drive = ((5e-4, 0.0, 0.0), (0.0, 0.0, 0.0))
    if name == "spheres128":
        shape = shape or (128, 128, 128)
        solid, info = sphere_pack(shape, 8.0 * shape[0] / 128.0, 0.40, seed=2207)
        xi = constant_xi(solid, xi45)
        steps = 5000
    elif name == "gauss256":
        shape = shape or (256, 256, 256)
        solid, info = gaussian_field_medium(shape, 4.0, 0.22, seed=1534)
        xi = constant_xi(solid, xi45)
        steps = 2000
    elif name == "spheres512":
        shape = shape or (512, 512, 512)
        solid, info = sphere_pack(shape, 12.0 * shape[0] / 512.0, 0.38, seed=512)
        xi = constant_xi(solid, xi45)
        steps = 1000
    elif name == "adjoint64":
        shape = shape or (64, 64, 64)
        solid, info = sphere_pack(shape, 6.0 * shape[0] / 64.0, 0.40, seed=64)
        xi = uniform_xi(solid, -0.4, 0.4, seed=6401)
        steps = 500
    else:
        raise ValueError(f"unknown workload {name!r}")
    rho = inlet_drainage_rho(solid)
    info["xi45"] = xi45
    info["xi45_cubic"] = xi_for_angle(45.0)
    return Workload(name, shape, solid, xi, rho, (1.5, 0.6), 3.5, g_drive, steps, info)
