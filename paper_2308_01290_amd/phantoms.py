"""Seeded synthetic inputs: ellipse phantoms, their exact fan-beam line
integrals, and Poisson noise.

This module is shared by the HIP path and the FP64 oracle, so it holds none of
the method's arithmetic: no attenuation model, no decomposition, no
regulariser.  Attenuation values of each ellipse are passed in by the caller
(``mu_of``), which keeps the physics on the side that uses it.

What it stands in for: the paper measures on scanner-reconstructed phantom and
patient images (Section III); those data are not available, so slices are
synthesised with the material ranges of the tissue-characterisation tables
(Table I: bone, soft tissue, lung inserts) inside a water body.

Geometry convention (the same one both compute paths implement on their own):
image pixel (row i, column k) covers x in [x0 + k*dx, x0 + (k+1)*dx),
y in [y0 + i*dx, y0 + (i+1)*dx) with x0 = -n_x*dx/2, y0 = -n_y*dx/2.  View v
has angle theta = angle0 + v*arc/n_views; the source sits at
sid*(cos theta, sin theta); the flat detector is centred at
-(sdd - sid)*(cos theta, sin theta) with axis e = (-sin theta, cos theta); bin
j is centred at u_j = (j - (n_det - 1)/2)*pitch + offset along e.  Ray (v, j)
is the line from the source to that bin centre.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Sequence, Tuple

import numpy as np

WATER_Z = 7.42
WATER_RHO = 1.0


@dataclass
class FanGeometry:
    """Plain description of a 2-D fan-beam scan (mm, radians)."""
    n_x: int
    n_y: int
    pixel_mm: float
    n_views: int
    n_det: int
    sid_mm: float
    sdd_mm: float
    det_pitch_mm: float = 0.0       # 0 -> pitch that covers the image corners
    det_offset_mm: float = 0.0
    angle0_rad: float = 0.0
    arc_rad: float = 2.0 * math.pi

    def pitch(self) -> float:
        if self.det_pitch_mm > 0:
            return float(self.det_pitch_mm)
        r = 0.5 * self.pixel_mm * math.hypot(self.n_x, self.n_y)
        return 2.0 * self.sdd_mm * math.tan(math.asin(r / self.sid_mm)) / self.n_det

    def resolved(self) -> "FanGeometry":
        g = FanGeometry(**self.__dict__)
        g.det_pitch_mm = self.pitch()
        return g


@dataclass
class Ellipse:
    cx: float
    cy: float
    a: float          # semi-axis along the rotated x axis (mm)
    b: float          # semi-axis along the rotated y axis (mm)
    phi: float        # rotation (rad)
    Z: float
    rho_e: float
    label: str = ""


@dataclass
class Phantom:
    body: Ellipse
    inserts: List[Ellipse] = field(default_factory=list)

    def ellipses(self) -> List[Ellipse]:
        return [self.body] + list(self.inserts)


# --------------------------------------------------------------------------
# workload geometries
# --------------------------------------------------------------------------

def geometry_small() -> FanGeometry:
    """128x128 at 1 mm, 180 views over 360 deg, 256 bins, SID 1000, SDD 1500."""
    return FanGeometry(n_x=128, n_y=128, pixel_mm=1.0, n_views=180, n_det=256,
                       sid_mm=1000.0, sdd_mm=1500.0).resolved()


def geometry_slice512() -> FanGeometry:
    """512x512 at 0.8 mm, 720 views, 736 bins, same fan (SID 1000, SDD 1500)."""
    return FanGeometry(n_x=512, n_y=512, pixel_mm=0.8, n_views=720, n_det=736,
                       sid_mm=1000.0, sdd_mm=1500.0).resolved()


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------

def _place(rng, n, inside, r_of, sep, max_tries=200000):
    """Rejection-sample n non-overlapping bounding circles."""
    placed: List[Tuple[float, float, float]] = []
    tries = 0
    while len(placed) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("phantom placement failed; relax the constraints")
        r = r_of(len(placed))
        c = inside(r)
        if c is None:
            continue
        if all(math.hypot(c[0] - p[0], c[1] - p[1]) >= r + p[2] + sep for p in placed):
            placed.append((c[0], c[1], r))
    return placed


def phantom_disk_inserts(seed: int = 1290, radius: float = 56.0, n_inserts: int = 8,
                         semi=(4.0, 14.0), Z=(5.5, 20.0), rho=(0.2, 1.9),
                         sep: float = 2.0) -> Phantom:
    """Water disk with seeded random elliptical inserts (small workload)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = [(rng.uniform(*semi), rng.uniform(*semi), rng.uniform(0.0, math.pi))
            for _ in range(n_inserts)]

    def inside(r):
        lim = radius - sep - r
        if lim <= 0:
            return None
        x, y = rng.uniform(-lim, lim, size=2)
        return (x, y) if math.hypot(x, y) <= lim else None

    centres = _place(rng, n_inserts, inside, lambda i: max(axes[i][0], axes[i][1]), sep)
    ins = []
    for (a, b, phi), (cx, cy, _) in zip(axes, centres):
        ins.append(Ellipse(cx, cy, a, b, phi, float(rng.uniform(*Z)),
                           float(rng.uniform(*rho)), "insert"))
    body = Ellipse(0.0, 0.0, radius, radius, 0.0, WATER_Z, WATER_RHO, "water")
    return Phantom(body, ins)


def phantom_body_inserts(seed: int = 2308, body_ax=(180.0, 140.0),
                         n_bone: int = 15, n_soft: int = 15, n_lung: int = 10,
                         semi=(3.0, 18.0), sep: float = 2.0) -> Phantom:
    """Elliptical water body with bone-like, soft-tissue and lung inserts.

    Material ranges follow the tissue-characterisation table (Table I):
    bone-like Z 11-14 / rho_e 1.1-1.7, soft tissue Z 6.5-8 / rho_e 0.93-1.06,
    lung rho_e 0.2-0.4 / Z 7.5-8.0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = ["bone"] * n_bone + ["soft"] * n_soft + ["lung"] * n_lung
    n = len(kinds)
    axes = [(rng.uniform(*semi), rng.uniform(*semi), rng.uniform(0.0, math.pi))
            for _ in range(n)]
    A, B = body_ax

    def inside(r):
        ea, eb = A - sep - r, B - sep - r
        if ea <= 0 or eb <= 0:
            return None
        x = rng.uniform(-ea, ea)
        y = rng.uniform(-eb, eb)
        return (x, y) if (x / ea) ** 2 + (y / eb) ** 2 <= 1.0 else None

    # big inserts first so that rejection sampling converges quickly
    order = sorted(range(n), key=lambda i: -max(axes[i][0], axes[i][1]))
    centres = _place(rng, n, inside, lambda t: max(axes[order[t]][0], axes[order[t]][1]), sep)
    ins: List[Ellipse] = [None] * n  # type: ignore
    for t, i in enumerate(order):
        a, b, phi = axes[i]
        kind = kinds[i]
        if kind == "bone":
            z, r = rng.uniform(11.0, 14.0), rng.uniform(1.1, 1.7)
        elif kind == "soft":
            z, r = rng.uniform(6.5, 8.0), rng.uniform(0.93, 1.06)
        else:
            z, r = rng.uniform(7.5, 8.0), rng.uniform(0.2, 0.4)
        ins[i] = Ellipse(centres[t][0], centres[t][1], a, b, phi, float(z), float(r), kind)
    body = Ellipse(0.0, 0.0, A, B, 0.0, WATER_Z, WATER_RHO, "water")
    return Phantom(body, ins)


def phantom_water_disk(radius: float = 56.0) -> Phantom:
    return Phantom(Ellipse(0.0, 0.0, radius, radius, 0.0, WATER_Z, WATER_RHO, "water"), [])


# --------------------------------------------------------------------------
# exact line integrals of ellipses (pure geometry)
# --------------------------------------------------------------------------

def ray_endpoints(geom: FanGeometry):
    """Source positions [V,2] and bin centres [V,D,2] in mm (FP64)."""
    g = geom.resolved()
    v = np.arange(g.n_views, dtype=np.float64)
    th = g.angle0_rad + v * (g.arc_rad / g.n_views)
    c, s = np.cos(th), np.sin(th)
    src = np.stack([g.sid_mm * c, g.sid_mm * s], axis=-1)
    u = (np.arange(g.n_det, dtype=np.float64) - 0.5 * (g.n_det - 1)) * g.det_pitch_mm \
        + g.det_offset_mm
    dcx = -(g.sdd_mm - g.sid_mm) * c
    dcy = -(g.sdd_mm - g.sid_mm) * s
    bx = dcx[:, None] + u[None, :] * (-s)[:, None]
    by = dcy[:, None] + u[None, :] * c[:, None]
    return src, np.stack([bx, by], axis=-1)


def ellipse_chords(e: Ellipse, src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """Length (mm) of each line src->dst inside the ellipse, exact closed form.

    With the line p + t*q (|q| = 1) mapped to the ellipse's unit-circle frame,
    |p' + t q'|^2 = 1 is a quadratic in t whose root gap is 2*sqrt(disc)/|q'|^2.
    """
    d = dst - src
    n = np.linalg.norm(d, axis=-1, keepdims=True)
    q = d / n
    p = src - np.array([e.cx, e.cy])
    cph, sph = math.cos(e.phi), math.sin(e.phi)
    px = (p[..., 0] * cph + p[..., 1] * sph) / e.a
    py = (-p[..., 0] * sph + p[..., 1] * cph) / e.b
    qx = (q[..., 0] * cph + q[..., 1] * sph) / e.a
    qy = (-q[..., 0] * sph + q[..., 1] * cph) / e.b
    qq = qx * qx + qy * qy
    pq = px * qx + py * qy
    pp = px * px + py * py
    disc = pq * pq - qq * (pp - 1.0)
    return np.where(disc > 0.0, 2.0 * np.sqrt(np.maximum(disc, 0.0)) / qq, 0.0)


MuFn = Callable[[np.ndarray, np.ndarray], Tuple[np.ndarray, np.ndarray]]


def analytic_sinograms(ph: Phantom, geom: FanGeometry, mu_of: MuFn):
    """Noise-free line integrals p_L, p_H [V, D] (FP64) of the phantom.

    ``mu_of(Z, rho_e) -> (mu_low, mu_high)`` gives each material's linear
    attenuation in 1/mm at the two acquisition energies.  Inserts sit inside
    the body and do not overlap, so each insert adds (mu_insert - mu_body)
    times its chord.
    """
    src, dst = ray_endpoints(geom)
    srcb = np.broadcast_to(src[:, None, :], dst.shape)
    Zs = np.array([e.Z for e in ph.ellipses()])
    Rs = np.array([e.rho_e for e in ph.ellipses()])
    muL, muH = mu_of(Zs, Rs)
    muL = np.asarray(muL, dtype=np.float64)
    muH = np.asarray(muH, dtype=np.float64)
    pL = np.zeros(dst.shape[:2])
    pH = np.zeros(dst.shape[:2])
    for idx, e in enumerate(ph.ellipses()):
        ch = ellipse_chords(e, srcb, dst)
        if idx == 0:
            pL += muL[0] * ch
            pH += muH[0] * ch
        else:
            pL += (muL[idx] - muL[0]) * ch
            pH += (muH[idx] - muH[0]) * ch
    return pL, pH


def poisson_log(p: np.ndarray, I0: float, seed: int) -> np.ndarray:
    """Post-log noisy line integrals: Y ~ Poisson(I0 exp(-p)), Y <- max(Y, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Y = rng.poisson(I0 * np.exp(-p)).astype(np.float64)
    Y = np.maximum(Y, 1.0)
    return -np.log(Y / I0)


# --------------------------------------------------------------------------
# rasterisation (for tests that need per-pixel truth)
# --------------------------------------------------------------------------

def pixel_centres(geom: FanGeometry):
    g = geom
    x = (np.arange(g.n_x) - 0.5 * (g.n_x - 1)) * g.pixel_mm
    y = (np.arange(g.n_y) - 0.5 * (g.n_y - 1)) * g.pixel_mm
    return np.meshgrid(x, y)   # X[i, k], Y[i, k]


def _inside(e: Ellipse, X, Y):
    c, s = math.cos(e.phi), math.sin(e.phi)
    dx, dy = X - e.cx, Y - e.cy
    u = (dx * c + dy * s) / e.a
    w = (-dx * s + dy * c) / e.b
    return u * u + w * w <= 1.0


def label_map(ph: Phantom, geom: FanGeometry, supersample: int = 1) -> np.ndarray:
    """Fractional coverage [n_ellipses+1, n_y, n_x]; plane 0 is air.

    Each pixel is sampled on an s x s grid; plane e holds the fraction of
    samples whose innermost ellipse is e (body = 1, inserts 2..).
    """
    s = int(supersample)
    g = geom
    off = (np.arange(s) + 0.5) / s - 0.5
    X, Y = pixel_centres(g)
    n_e = len(ph.ellipses())
    out = np.zeros((n_e + 1, g.n_y, g.n_x))
    for ox in off:
        for oy in off:
            Xs, Ys = X + ox * g.pixel_mm, Y + oy * g.pixel_mm
            lab = np.zeros(X.shape, dtype=np.int64)
            for idx, e in enumerate(ph.ellipses()):
                lab[_inside(e, Xs, Ys)] = idx + 1
            for idx in range(n_e + 1):
                out[idx] += (lab == idx)
    return out / (s * s)


def material_maps(ph: Phantom, geom: FanGeometry, supersample: int = 1):
    """Coverage-weighted per-pixel (Z, rho_e) maps; air is (0, 0)."""
    lab = label_map(ph, geom, supersample)
    Z = np.zeros(lab.shape[1:])
    R = np.zeros(lab.shape[1:])
    for idx, e in enumerate(ph.ellipses()):
        Z += lab[idx + 1] * e.Z
        R += lab[idx + 1] * e.rho_e
    return Z, R, lab


def mu_maps(ph: Phantom, geom: FanGeometry, mu_of: MuFn, supersample: int = 1):
    """Coverage-weighted per-pixel attenuation images (mu_L, mu_H) in 1/mm."""
    lab = label_map(ph, geom, supersample)
    Zs = np.array([e.Z for e in ph.ellipses()])
    Rs = np.array([e.rho_e for e in ph.ellipses()])
    muL, muH = mu_of(Zs, Rs)
    iL = np.zeros(lab.shape[1:])
    iH = np.zeros(lab.shape[1:])
    for idx in range(len(Zs)):
        iL += lab[idx + 1] * muL[idx]
        iH += lab[idx + 1] * muH[idx]
    return iL, iH


def workload_small(mu_of: MuFn, seed: int = 1290, noise_seeds=(1291, 1292), I0=(1e5, 1e5)):
    """Small workload: 128^2 water disk with 8 random inserts, Poisson 1e5."""
    geom = geometry_small()
    ph = phantom_disk_inserts(seed)
    pL, pH = analytic_sinograms(ph, geom, mu_of)
    return geom, ph, poisson_log(pL, I0[0], noise_seeds[0]), poisson_log(pH, I0[1], noise_seeds[1])


def workload_slice512(mu_of: MuFn, seed: int = 2308, noise_seeds=(2309, 2310), I0=(5e4, 1e5)):
    """512^2 slice: elliptical body with 40 inserts, Poisson 5e4 (low) / 1e5 (high)."""
    geom = geometry_slice512()
    ph = phantom_body_inserts(seed)
    pL, pH = analytic_sinograms(ph, geom, mu_of)
    return geom, ph, poisson_log(pL, I0[0], noise_seeds[0]), poisson_log(pH, I0[1], noise_seeds[1])


# --------------------------------------------------------------------------
# batches of uneven slices
# --------------------------------------------------------------------------
UNEVEN_SIZES = (256, 384, 512)
UNEVEN_VIEWS = (360, 720, 984)
UNEVEN_BINS = (512, 888)


def geometry_uneven(seed: int) -> FanGeometry:
    """One slice of an uneven batch: n in {256, 384, 512} at 0.8 mm, views in
    {360, 720, 984} over 360 deg, bins uniform in 512..888, SID 1000, SDD 1500."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.choice(UNEVEN_SIZES))
    v = int(rng.choice(UNEVEN_VIEWS))
    d = int(rng.integers(UNEVEN_BINS[0], UNEVEN_BINS[1] + 1))
    return FanGeometry(n_x=n, n_y=n, pixel_mm=0.8, n_views=v, n_det=d, sid_mm=1000.0,
                       sdd_mm=1500.0).resolved()


def slice_uneven(seed: int, mu_of: MuFn, I0=(5e4, 1e5)):
    """(geometry, phantom, p_lo, p_hi) of uneven-batch slice `seed`: the body
    phantom of the 512^2 slice scaled to the slice's field of view."""
    geom = geometry_uneven(seed)
    s = geom.n_x / 512.0
    ph = phantom_body_inserts(seed, body_ax=(180.0 * s, 140.0 * s), semi=(3.0 * s, 18.0 * s))
    pL, pH = analytic_sinograms(ph, geom, mu_of)
    return (geom, ph, poisson_log(pL, I0[0], 2 * seed + 1), poisson_log(pH, I0[1], 2 * seed + 2))


def workload_uneven(mu_of: MuFn, n_slices: int = 64, seed0: int = 3000):
    """The uneven batch: slices seed0, seed0 + 1, ... (list of slice_uneven tuples)."""
    return [slice_uneven(seed0 + i, mu_of) for i in range(n_slices)]


# --------------------------------------------------------------------------
# single-slice serving requests
# --------------------------------------------------------------------------
SERVE_SIZES = (256, 384, 512, 768)


def geometry_served(n: int, seed: int, n_views=None, n_det=None) -> FanGeometry:
    """Geometry of a served request: image n at 0.8 mm, views uniform in
    360..1152 and bins uniform in 512..1024 drawn from the seed (or given)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = int(rng.integers(360, 1153))
    d = int(rng.integers(512, 1025))
    return FanGeometry(n_x=n, n_y=n, pixel_mm=0.8, n_views=n_views or v, n_det=n_det or d,
                       sid_mm=1000.0, sdd_mm=1500.0).resolved()


def slice_served(n: int, seed: int, mu_of: MuFn, n_views=None, n_det=None, I0=(5e4, 1e5)):
    """(geometry, phantom, p_lo, p_hi) of a served request: the body phantom of
    the 512^2 slice scaled to the field of view, Poisson 5e4 / 1e5."""
    geom = geometry_served(n, seed, n_views, n_det)
    s = n / 512.0
    ph = phantom_body_inserts(seed, body_ax=(180.0 * s, 140.0 * s), semi=(3.0 * s, 18.0 * s))
    pL, pH = analytic_sinograms(ph, geom, mu_of)
    return geom, ph, poisson_log(pL, I0[0], 2 * seed + 1), poisson_log(pH, I0[1], 2 * seed + 2)


# --------------------------------------------------------------------------
# image-domain inputs (attenuation image pairs)
# --------------------------------------------------------------------------
# Relative noise of the two attenuation images, in units of water's
# attenuation at each energy: the per-pixel noise level of a clinical
# reconstruction (about 15 and 10 HU).
IMAGE_NOISE_REL = (0.015, 0.010)


def noisy_mu_pair(ph: Phantom, geom: FanGeometry, mu_of: MuFn, seed: int,
                  rel=IMAGE_NOISE_REL, supersample: int = 2):
    """(mu_L, mu_H) of a phantom on the image grid (coverage-weighted, 2x2
    supersampled) plus independent white Gaussian noise of standard deviation
    rel[k] * mu_water(E_k), seeded."""
    muL, muH = mu_maps(ph, geom, mu_of, supersample)
    wL, wH = mu_of(np.array([WATER_Z]), np.array([WATER_RHO]))
    rng = np.random.default_rng(seed)
    nL = rng.standard_normal(muL.shape) * (rel[0] * float(wL[0]))
    nH = rng.standard_normal(muH.shape) * (rel[1] * float(wH[0]))
    return muL + nL, muH + nH


def workload_image_small(mu_of: MuFn, seed: int = 1290, noise_seed: int = 1293):
    """128^2 / 1 mm water disk with 8 inserts (the small phantom) as noisy
    attenuation images."""
    geom = geometry_small()
    ph = phantom_disk_inserts(seed)
    muL, muH = noisy_mu_pair(ph, geom, mu_of, noise_seed)
    return geom, ph, muL, muH


def workload_image512(mu_of: MuFn, seed: int = 2308, noise_seed: int = 2311):
    """512^2 / 0.8 mm body with 40 inserts (the 512^2 slice's phantom) as noisy
    attenuation images."""
    geom = geometry_slice512()
    ph = phantom_body_inserts(seed)
    muL, muH = noisy_mu_pair(ph, geom, mu_of, noise_seed)
    return geom, ph, muL, muH
