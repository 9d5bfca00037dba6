"""Seeded synthetic inputs for the PSL dose path.

This module is the only code shared by the oracle and the HIP path.  It
draws inputs (phase spaces, bin grids, phantoms, jaw settings, fluence maps,
treatment plans) and holds none of the method's arithmetic: no binning, no
culling, no allocation, no sampling, no transport, no tally.

The paper's data (a BEAMnrc phase space of a 6 MV Clinac 21EX and a patient
CT, Sec. 2.6) are not available; every generator here is a seeded stand-in
with the shapes and distributions of the workloads described in the paper's
testing cases (Sec. 2.6) and the five workload definitions listed in
``WORKLOADS``.

Coordinates: beam frame, cm.  The source (target) sits at the origin and the
beam travels along +z.  The isocentre is at z = SAD = 100 cm.  Energies are
kinetic, in MeV.  Particle type 0 = photon, 1 = electron or positron
(merged, Sec. 2.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# ----------------------------------------------------------------------------
# Geometry constants (beam frame, cm).  The paper gives SAD = 100 cm and an
# SSD of 90 cm for its water tests (Sec. 2.6); it does not give the heights of
# the PSL plane or of the jaws, so these are stated readings.
# ----------------------------------------------------------------------------
SAD = 100.0
Z_PSL = 25.0        # PSL (phase-space) plane
Z_JAW_Y = 28.0      # upper jaw pair (Y)
Z_JAW_X = 37.0      # lower jaw pair (X)

# Physics constants of the transport model (water, Compton-only photons,
# CSDA electrons with Bethe collision stopping power).
ELECTRON_DENSITY_WATER = 3.343e23   # electrons / cm^3 at 1 g/cm^3
MEAN_EXCITATION_EV = 75.0
RADIATION_LENGTH_WATER = 36.08      # g/cm^2
STEP_CM = 0.1                       # 1 mm electron step
PHOTON_CUTOFF = 0.010               # MeV (Sec. 2.6)
ELECTRON_CUTOFF = 0.700 - 0.51099895  # MeV kinetic; 0.700 MeV total (Sec. 2.6)


@dataclasses.dataclass
class PhaseSpace:
    """Structure-of-arrays phase space at the plane z = z_plane."""
    type: np.ndarray   # uint8
    E: np.ndarray      # float32, kinetic MeV
    x: np.ndarray      # float32, cm
    y: np.ndarray
    u: np.ndarray      # float32 direction cosines
    v: np.ndarray
    w: np.ndarray
    wt: np.ndarray     # float32 statistical weight
    z_plane: float

    @property
    def n(self) -> int:
        return int(self.E.shape[0])

    def fields(self):
        return ("type", "E", "x", "y", "u", "v", "w", "wt")

    def subset(self, idx) -> "PhaseSpace":
        return PhaseSpace(*(getattr(self, f)[idx] for f in self.fields()),
                          z_plane=self.z_plane)


def phase_space(n: int, seed: int, half_width: float, z_plane: float,
                p_electron: float = 0.03, e_min: float = 0.1,
                e_mode: float = 1.0, e_max: float = 6.0,
                sigma_src: float = 0.1, z_aim: float = SAD,
                aim: str = "square") -> PhaseSpace:
    """Linac-like synthetic phase space.

    Particles leave a Gaussian point source (sigma ``sigma_src`` cm in x and
    y) at z = 0, aimed at a point drawn uniformly over the square
    [-half_width, half_width)^2 at z = ``z_aim`` (aim="square"), or over the
    disk of radius half_width (aim="disk": a cylindrically symmetric phase
    space, for azimuthal redistribution).  Each is recorded where its ray
    crosses z = ``z_plane``.  A fraction ``p_electron`` are electrons;
    energies follow a triangular spectrum (e_min, e_mode, e_max).  Weights
    are 1.
    """
    rng = np.random.default_rng(seed)
    t = (rng.random(n) < p_electron).astype(np.uint8)
    E = rng.triangular(e_min, e_mode, e_max, n)
    sx = rng.normal(0.0, sigma_src, n)
    sy = rng.normal(0.0, sigma_src, n)
    if aim == "disk":
        rad = half_width * np.sqrt(rng.random(n))
        ang = rng.uniform(0.0, 2.0 * np.pi, n)
        ax, ay = rad * np.cos(ang), rad * np.sin(ang)
    else:
        ax = rng.uniform(-half_width, half_width, n)
        ay = rng.uniform(-half_width, half_width, n)
    dx, dy, dz = ax - sx, ay - sy, np.full(n, z_aim)
    norm = np.sqrt(dx * dx + dy * dy + dz * dz)
    u, v, w = dx / norm, dy / norm, dz / norm
    frac = z_plane / z_aim
    x = sx + dx * frac
    y = sy + dy * frac
    f32 = np.float32
    return PhaseSpace(t, E.astype(f32), x.astype(f32), y.astype(f32),
                      u.astype(f32), v.astype(f32), w.astype(f32),
                      np.ones(n, f32), float(z_plane))


@dataclasses.dataclass
class Grid:
    """PSL bin grid: energy edges and position edges at z_plane (float32)."""
    e_edges: np.ndarray
    x_edges: np.ndarray
    y_edges: np.ndarray
    z_plane: float

    @property
    def n_e(self):
        return len(self.e_edges) - 1

    @property
    def n_x(self):
        return len(self.x_edges) - 1

    @property
    def n_y(self):
        return len(self.y_edges) - 1

    @property
    def n_keys(self):
        return 2 * self.n_e * self.n_x * self.n_y


def linear_edges(lo: float, hi: float, n: int) -> np.ndarray:
    """n uniform bins on [lo, hi]; edge k = lo + k (hi - lo) / n in double,
    rounded once to float32."""
    k = np.arange(n + 1, dtype=np.float64)
    e = lo + k * (hi - lo) / n
    e[-1] = hi
    return e.astype(np.float32)


def log_edges(lo: float, hi: float, n: int) -> np.ndarray:
    """n log-spaced bins on [lo, hi]; edge k = lo (hi/lo)^(k/n), rounded to
    float32."""
    k = np.arange(n + 1, dtype=np.float64)
    e = lo * (hi / lo) ** (k / n)
    e[0], e[-1] = lo, hi
    return e.astype(np.float32)


@dataclasses.dataclass
class Phantom:
    """Voxel phantom; density[iz, iy, ix] in g/cm^3, x fastest in memory."""
    density: np.ndarray     # float32 (nz, ny, nx)
    voxel: tuple            # (dx, dy, dz) cm
    origin: tuple           # (x0, y0, z0) cm, corner of voxel (0,0,0)

    @property
    def shape(self):
        return self.density.shape


def water_phantom(n: tuple, voxel: float, origin: tuple) -> Phantom:
    nx, ny, nz = n
    return Phantom(np.ones((nz, ny, nx), np.float32), (voxel,) * 3,
                   tuple(float(o) for o in origin))


def heterogeneous_phantom(n: tuple, voxel: float, origin: tuple, seed: int,
                          n_lung: int = 2, n_bone: int = 2) -> Phantom:
    """Water with lung ellipsoids (0.26 g/cm^3) and bone slabs normal to z
    (1.85 g/cm^3); bone overrides lung overrides water."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    x0, y0, z0 = origin
    xc = x0 + (np.arange(nx) + 0.5) * voxel
    yc = y0 + (np.arange(ny) + 0.5) * voxel
    zc = z0 + (np.arange(nz) + 0.5) * voxel
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    rho = np.ones((nz, ny, nx), np.float32)
    lx, ly, lz = nx * voxel, ny * voxel, nz * voxel
    for _ in range(n_lung):
        a = rng.uniform(2.0, 6.0, 3)
        c = np.array([x0 + rng.uniform(0.25, 0.75) * lx,
                      y0 + rng.uniform(0.25, 0.75) * ly,
                      z0 + rng.uniform(0.25, 0.75) * lz])
        inside = (((X - c[0]) / a[0]) ** 2 + ((Y - c[1]) / a[1]) ** 2
                  + ((Z - c[2]) / a[2]) ** 2) <= 1.0
        rho[inside] = 0.26
    for _ in range(n_bone):
        th = rng.uniform(0.5, 2.0)
        zs = z0 + rng.uniform(0.1, 0.9) * (lz - th)
        rho[(Z >= zs) & (Z < zs + th)] = 1.85
    return Phantom(rho, (voxel,) * 3, tuple(float(o) for o in origin))


@dataclasses.dataclass
class Field:
    """One field (or IMRT segment).  Jaw edges are given as their projection
    at the SAD plane, in cm.  ``fluence`` is a (nfy, nfx) float32 map defined
    at the SAD plane, pixel (j, i) covering [f_x0 + i pix, f_x0 + (i+1) pix)
    x [f_y0 + j pix, ...); None means no modulation."""
    X1: float
    X2: float
    Y1: float
    Y2: float
    gantry_deg: float = 0.0
    MU: float = 1.0
    fluence: Optional[np.ndarray] = None
    f_x0: float = -20.0
    f_y0: float = -20.0
    f_pix: float = 1.0
    jaws: bool = True
    collimator_deg: float = 0.0
    couch_deg: float = 0.0


def square_field(side: float, MU: float = 1.0) -> Field:
    h = side / 2.0
    return Field(-h, h, -h, h, MU=MU)


def fluence_map(seed: int, n: int = 40) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((n, n)).astype(np.float32)


def random_jaws(seed: int, lim: float = 15.0, min_open: float = 1.0):
    rng = np.random.default_rng(seed)
    while True:
        xs = np.sort(rng.uniform(-lim, lim, 2))
        ys = np.sort(rng.uniform(-lim, lim, 2))
        if xs[1] - xs[0] >= min_open and ys[1] - ys[0] >= min_open:
            return float(xs[0]), float(xs[1]), float(ys[0]), float(ys[1])


def imrt_plan(seed: int, n_beams: int = 7, n_segments: int = 20,
              lim: float = 15.0) -> List[Field]:
    """Coplanar beams at gantry 360 k / n_beams, each with ``n_segments``
    rectangular apertures with sides U[1, 20] cm whose edges stay within
    +-lim, a per-segment U[0,1] 40x40 fluence map and MU ~ U[1, 100]."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_beams):
        g = 360.0 * b / n_beams
        for s in range(n_segments):
            wx, wy = rng.uniform(1.0, 20.0, 2)
            cx = rng.uniform(-lim + wx / 2, lim - wx / 2)
            cy = rng.uniform(-lim + wy / 2, lim - wy / 2)
            fl = rng.random((40, 40)).astype(np.float32)
            mu = float(rng.uniform(1.0, 100.0))
            out.append(Field(cx - wx / 2, cx + wx / 2, cy - wy / 2,
                             cy + wy / 2, gantry_deg=g, MU=mu, fluence=fl))
    return out


def vmat_plan(seed: int, arcs=((0.0, 360.0, 30.0, 0.0),
                                (90.0, 270.0, 330.0, 90.0)),
              step_deg: float = 4.0, lim: float = 12.0) -> List[Field]:
    """Arcs as many control points (Sec. 2.4: one fluence map per beam
    angle).  Each arc (gantry start, gantry stop, collimator, couch) gets a
    control point every step_deg degrees of gantry; a control point has
    jaws that follow a slowly moving aperture (sides 4-16 cm, edges within
    +-lim), a 40x40 fluence map of its own (a smooth field times U[0.5, 1]
    noise) and MU ~ U[0.5, 2]."""
    rng = np.random.default_rng(seed)
    out = []
    for g0, g1, coll, couch in arcs:
        n = int(round((g1 - g0) / step_deg))
        phase = rng.uniform(0, 2 * np.pi, 4)
        for k in range(n):
            g = (g0 + k * step_deg) % 360.0
            a = 2 * np.pi * k / max(n, 1)
            wx = 10.0 + 6.0 * np.sin(a + phase[0])
            wy = 10.0 + 6.0 * np.sin(a + phase[1])
            cx = (lim - wx / 2) * 0.5 * np.sin(2 * a + phase[2])
            cy = (lim - wy / 2) * 0.5 * np.sin(2 * a + phase[3])
            yy, xx = np.mgrid[0:40, 0:40]
            smooth = 0.5 + 0.5 * np.cos((xx - 20) / 40.0 * np.pi * (1 + k % 3)) \
                * np.cos((yy - 20) / 40.0 * np.pi)
            fl = (smooth * rng.uniform(0.5, 1.0, (40, 40))).astype(np.float32)
            out.append(Field(cx - wx / 2, cx + wx / 2, cy - wy / 2,
                             cy + wy / 2, gantry_deg=g,
                             MU=float(rng.uniform(0.5, 2.0)), fluence=fl,
                             collimator_deg=coll, couch_deg=couch))
    return out


# ----------------------------------------------------------------------------
# The five workloads.  Seeds: inputs 1000 + workload number, transport
# 2000 + workload number (batch b adds b).
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    phsp: PhaseSpace
    grid: Grid
    phantom: Phantom
    fields: List[Field]
    histories: int          # total per field set (all batches)
    batches: int
    fixed_point: bool       # 64-bit fixed-point tally (else FP64)
    cull: bool
    alloc_mode: int         # 0: proportional to selected counts; 1: to MU
    seed: int


def workload_tiny(n_particles: int = 100_000, histories: int = 1_000_000,
                  batches: int = 10) -> Workload:
    """Plain method, tiny: 1e5 particles aimed over 10x10 cm at the surface
    of a 30 cm water cube (60^3, 5 mm) at SSD 100; 16 linear energy bins,
    1 cm position grid, recorded at the surface; FP64 tally; no jaws."""
    ps = phase_space(n_particles, 1001, 5.0, SAD)
    emax = float(ps.E.max())
    g = Grid(linear_edges(0.0, emax, 16), linear_edges(-5.0, 5.0, 10),
             linear_edges(-5.0, 5.0, 10), SAD)
    ph = water_phantom((60, 60, 60), 0.5, (-15.0, -15.0, SAD))
    f = Field(-5.0, 5.0, -5.0, 5.0, jaws=False)
    return Workload("tiny-water-60", ps, g, ph, [f], histories, batches,
                    False, False, 0, 2001)


def clinical_grid() -> Grid:
    return Grid(log_edges(0.1, 6.0, 32), linear_edges(-5.5, 5.5, 22),
                linear_edges(-5.5, 5.5, 22), Z_PSL)


def workload_clinical(side: float = 10.0, n_particles: int = 10_000_000,
                      histories: int = 100_000_000,
                      batches: int = 10) -> Workload:
    """PSL at clinical scale: 1e7 particles aimed over 40x40 cm at the SAD
    plane, recorded at the PSL plane; 32 log energy bins, 5 mm position
    bins; square open field; 128^3 water at 2.5 mm, SSD 100; fixed-point
    tally."""
    ps = phase_space(n_particles, 1002, 20.0, Z_PSL)
    ph = water_phantom((128, 128, 128), 0.25, (-16.0, -16.0, SAD))
    return Workload(f"clinical-{side:g}x{side:g}-water-128", ps,
                    clinical_grid(), ph, [square_field(side)], histories,
                    batches, True, True, 0, 2002)


def workload_heterogeneous(n_particles: int = 10_000_000,
                           histories: int = 300_000_000,
                           batches: int = 10,
                           shape=(256, 256, 160), voxel=0.2) -> Workload:
    """Random jaws within +-15 cm, a 40x40 U[0,1] fluence map and a
    heterogeneous 256x256x160 phantom at 2 mm."""
    ps = phase_space(n_particles, 1002, 20.0, Z_PSL)
    X1, X2, Y1, Y2 = random_jaws(1003)
    f = Field(X1, X2, Y1, Y2, fluence=fluence_map(1003))
    nx, ny, nz = shape
    ph = heterogeneous_phantom(shape, voxel,
                               (-nx * voxel / 2, -ny * voxel / 2, SAD), 1003)
    return Workload("heterogeneous-256x256x160", ps, clinical_grid(), ph,
                    [f], histories, batches, True, True, 0, 2003)


def workload_vmat(n_particles: int = 10_000_000,
                  histories: int = 1_000_000_000,
                  batches: int = 10, step_deg: float = 4.0) -> Workload:
    """Two arcs as control points on the 128^3 water phantom centred on
    the isocentre: a coplanar 360-degree arc at collimator 30, and a
    non-coplanar 180-degree arc at couch 90 and collimator 330 (135 control
    points at 4 degrees); histories proportional to MU."""
    ps = phase_space(n_particles, 1002, 20.0, Z_PSL)
    ph = water_phantom((128, 128, 128), 0.25, (-16.0, -16.0, SAD - 16.0))
    return Workload("vmat-2arcs-water-128", ps, clinical_grid(), ph,
                    vmat_plan(1006, step_deg=step_deg), histories, batches,
                    True, True, 1, 2006)


def workload_imrt(n_particles: int = 10_000_000,
                  histories: int = 1_000_000_000,
                  batches: int = 10) -> Workload:
    """7 coplanar beams x 20 segments on the 128^3 water phantom centred on
    the isocentre; histories proportional to MU."""
    ps = phase_space(n_particles, 1002, 20.0, Z_PSL)
    ph = water_phantom((128, 128, 128), 0.25, (-16.0, -16.0, SAD - 16.0))
    return Workload("imrt-7x20-water-128", ps, clinical_grid(), ph,
                    imrt_plan(1004), histories, batches, True, True, 1, 2004)
