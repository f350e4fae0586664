"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module only *generates inputs*: velocity models, acquisition geometry
and the source wavelet.  It holds none of the method's arithmetic (no
stencil, no sponge, no adjoint, no Anderson step), so that the oracle and
the GPU path can both consume it without sharing any of the computation
they are compared on.

Every array that crosses into a solver is rounded to FP32 once, here, so
that both sides start from bit-identical inputs.

Seeds follow ``numpy.random.default_rng(1000*config + 10*instance +
purpose)`` with purpose codes 0 layers/velocities, 1 anomalies/reflectors,
2 texture, 3 faults, 4 noise, 5 CNN init, 6 training order.

The paper's own workloads (a 3 x 9 km section with a 4 s record, Section
"Numerical Example") are stood in for by the seeded models below; no values
of any public benchmark model are reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.ndimage import gaussian_filter

__all__ = [
    "Geometry", "ricker", "make_geometry", "seed", "linear_gaussian_model",
    "layered_model", "smooth", "lsrtm_background", "sparse_reflectors",
    "config1", "config2", "config3", "config4_instances", "config5",
    "learned_instance", "small_case", "uniform_noise",
]

PURPOSE_LAYERS, PURPOSE_ANOMALY, PURPOSE_TEXTURE, PURPOSE_FAULTS, \
    PURPOSE_NOISE, PURPOSE_CNN_INIT, PURPOSE_TRAIN_ORDER = range(7)


def seed(config: int, instance: int, purpose: int) -> np.random.Generator:
    return np.random.default_rng(1000 * config + 10 * instance + purpose)


@dataclasses.dataclass
class Geometry:
    """Acquisition and grid description (host memory, plain numbers).

    Interior grid ``nz x nx`` with spacing ``h`` (dx = dz); ``nb`` sponge
    cells on all four sides; ``nt`` time steps of ``dt``.  Sources and
    receivers are interior node indices.  ``vref`` is the fixed velocity the
    sponge strength is computed from; ``refl`` its nominal reflection
    coefficient.  ``vmax_bound`` is the largest velocity the caller promises
    the model will ever hold (the CFL check uses it).
    """
    nz: int
    nx: int
    h: float
    nb: int
    dt: float
    nt: int
    vref: float
    refl: float
    vmax_bound: float
    src_iz: np.ndarray  # int32 [S]
    src_ix: np.ndarray  # int32 [S]
    rec_iz: np.ndarray  # int32 [S, R]
    rec_ix: np.ndarray  # int32 [S, R]
    wavelet: np.ndarray  # float32 [nt]

    @property
    def nshots(self) -> int:
        return int(self.src_iz.shape[0])

    @property
    def nrec(self) -> int:
        return int(self.rec_iz.shape[1])

    @property
    def nz_p(self) -> int:
        return self.nz + 2 * self.nb

    @property
    def nx_p(self) -> int:
        return self.nx + 2 * self.nb

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)

    def subset_shots(self, shots) -> "Geometry":
        shots = np.asarray(shots)
        return self.replace(src_iz=self.src_iz[shots].copy(), src_ix=self.src_ix[shots].copy(),
                            rec_iz=self.rec_iz[shots].copy(), rec_ix=self.rec_ix[shots].copy())


def ricker(nt: int, dt: float, f0: float) -> np.ndarray:
    """Ricker wavelet with unit peak, delayed by 1.5/f0, sampled at n*dt."""
    t = np.arange(nt, dtype=np.float64) * dt - 1.5 / f0
    a = (math.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def make_geometry(nz, nx, h, nt, dt, nshots, rec_stride=1, f0=10.0, nb=20,
                  src_depth=2, rec_depth=2, vref=3000.0, vmax_bound=None,
                  refl=1e-3) -> Geometry:
    """Equally spaced surface shots; receivers on every ``rec_stride`` column."""
    src_ix = np.array([int(round((i + 0.5) * nx / nshots)) for i in range(nshots)], dtype=np.int32)
    src_ix = np.clip(src_ix, 0, nx - 1).astype(np.int32)
    src_iz = np.full(nshots, src_depth, dtype=np.int32)
    cols = np.arange(0, nx, rec_stride, dtype=np.int32)
    rec_ix = np.tile(cols, (nshots, 1)).astype(np.int32)
    rec_iz = np.full_like(rec_ix, rec_depth)
    if vmax_bound is None:
        vmax_bound = 0.5 * h / dt
    return Geometry(nz=nz, nx=nx, h=float(h), nb=nb, dt=float(dt), nt=nt, vref=float(vref),
                    refl=float(refl), vmax_bound=float(vmax_bound), src_iz=src_iz,
                    src_ix=src_ix, rec_iz=rec_iz, rec_ix=rec_ix,
                    wavelet=ricker(nt, dt, f0))


def smooth(v: np.ndarray, sigma_cells: float) -> np.ndarray:
    return gaussian_filter(np.asarray(v, np.float64), sigma=sigma_cells, mode="nearest")


def to_m(v: np.ndarray) -> np.ndarray:
    """Squared slowness m = 1/v^2 as the FP32 array both sides receive."""
    return (1.0 / np.asarray(v, np.float64) ** 2).astype(np.float32)


def linear_gaussian_model(nz, nx, rng, v_top=2000.0, v_bot=3000.0, amp=200.0,
                          sigma_cells=8.0):
    """Linear v(z) plus one positive and one negative Gaussian anomaly."""
    iz = np.arange(nz, dtype=np.float64)[:, None]
    ix = np.arange(nx, dtype=np.float64)[None, :]
    v = v_top + (v_bot - v_top) * iz / (nz - 1) + 0.0 * ix
    for sign in (+1.0, -1.0):
        cz = rng.uniform(0.25 * nz, 0.75 * nz)
        cx = rng.uniform(0.1875 * nx, 0.8125 * nx)
        v = v + sign * amp * np.exp(-((iz - cz) ** 2 + (ix - cx) ** 2) / (2 * sigma_cells ** 2))
    return v


def layered_model(nz, nx, h, config, instance, nlayers=12, v_top=1500.0, v_bot=5500.0,
                  texture_std=50.0):
    """Dipping layers with two faults and Gaussian texture."""
    rl = seed(config, instance, PURPOSE_LAYERS)
    vel = np.linspace(v_top, v_bot, nlayers)
    vel[1:-1] += rl.uniform(-100.0, 100.0, nlayers - 2)
    vel = np.sort(vel)
    depth = nz * h
    base = np.linspace(0.08, 0.95, nlayers - 1) * depth
    base = base + rl.uniform(-0.02, 0.02, nlayers - 1) * depth
    dip0 = rl.uniform(-8.0, 8.0)
    dips = dip0 + rl.uniform(-2.0, 2.0, nlayers - 1)
    z = (np.arange(nz) + 0.5)[:, None] * h
    x = (np.arange(nx) + 0.5)[None, :] * h
    xc = 0.5 * nx * h
    # fault throws: the hanging wall sees the interfaces shifted down
    rf = seed(config, instance, PURPOSE_FAULTS)
    shift = np.zeros((nz, nx))
    for _ in range(2):
        fx, fz = rf.uniform(0.15, 0.85) * nx * h, rf.uniform(0.2, 0.8) * depth
        ang = math.radians(rf.uniform(60.0, 80.0)) * (1 if rf.uniform() < 0.5 else -1)
        throw = rf.uniform(25.0, 100.0)
        # signed side of the fault line through (fx, fz) with angle ang from horizontal
        side = (x - fx) * math.sin(ang) - (z - fz) * math.cos(ang)
        shift = shift + np.where(side > 0, throw, 0.0)
    zz = z - shift
    layer = np.zeros((nz, nx), dtype=np.int64)
    for i in range(nlayers - 1):
        iface = base[i] + np.tan(np.radians(dips[i])) * (x - xc)
        layer += (zz > iface).astype(np.int64)
    v = vel[layer]
    rt = seed(config, instance, PURPOSE_TEXTURE)
    tex = gaussian_filter(rt.standard_normal((nz, nx)), sigma=2.0, mode="nearest")
    tex *= texture_std / max(tex.std(), 1e-30)
    return np.clip(v + tex, 1450.0, 5600.0)


def lsrtm_background(nz, nx, v_top=1500.0, v_bot=4500.0):
    iz = np.arange(nz, dtype=np.float64)[:, None]
    return np.repeat(v_top + (v_bot - v_top) * iz / (nz - 1), nx, axis=1)


def sparse_reflectors(m0: np.ndarray, config, instance, nref=40, amp_std=0.05):
    """Relative perturbation dm = a * m0 on one-cell-thick dipping segments."""
    nz, nx = m0.shape
    r = seed(config, instance, PURPOSE_ANOMALY)
    dm = np.zeros((nz, nx))
    for _ in range(nref):
        cz = r.uniform(min(16, nz - 1), nz - 1)
        cx = r.uniform(0, nx - 1)
        length = r.uniform(40, 200) * nx / 768.0
        dip = math.radians(r.uniform(-15.0, 15.0))
        a = r.normal(0.0, amp_std)
        for t in np.linspace(-0.5 * length, 0.5 * length, int(max(2, length * 2))):
            ix = int(round(cx + t * math.cos(dip)))
            iz = int(round(cz + t * math.sin(dip)))
            if 0 <= ix < nx and 0 <= iz < nz:
                dm[iz, ix] = a * m0[iz, ix]
    return dm.astype(np.float32)


def config1():
    """128x128, 10 m, 800 steps, 4 shots, 128 receivers; linear v(z) + anomalies."""
    nz = nx = 128
    g = make_geometry(nz, nx, 10.0, 800, 1e-3, 4, rec_stride=1, vref=3000.0)
    v_true = linear_gaussian_model(nz, nx, seed(1, 0, PURPOSE_ANOMALY))
    v0 = smooth(v_true, 10.0)
    g = g.replace(vref=float(v0.max()))
    return g, to_m(v_true), to_m(v0)


def config2(nshots=64, nt=4000):
    """768x256 (nx x nz), 12.5 m, 4000 steps, 64 shots, 384 receivers; layered model."""
    nz, nx, h = 256, 768, 12.5
    g = make_geometry(nz, nx, h, nt, 1e-3, nshots, rec_stride=2)
    v_true = layered_model(nz, nx, h, 2, 0)
    v0 = smooth(v_true, 8.0)
    g = g.replace(vref=float(v0.max()))
    return g, to_m(v_true), to_m(v0)


def config3(nshots=64, nt=4000):
    """LSRTM: smooth v(z) 1500->4500 background and 40 sparse reflectors."""
    nz, nx, h = 256, 768, 12.5
    g = make_geometry(nz, nx, h, nt, 1e-3, nshots, rec_stride=2)
    v0 = lsrtm_background(nz, nx)
    m0 = to_m(v0)
    dm = sparse_reflectors(m0.astype(np.float64), 3, 0)
    g = g.replace(vref=float(v0.max()))
    return g, m0, dm


def config4_instances(ninst=32, first=0):
    """Uneven batch: grid, spacing, record length and shot count drawn per
    instance; instances first, first + 1, ... (the batched workload uses
    0 .. 31; further instances of the same family start at 100)."""
    grids = [(128, 128), (256, 128), (384, 128), (512, 256), (768, 256), (1024, 384), (1024, 512)]
    hs = [10.0, 12.5, 15.0, 20.0]
    out = []
    for i in range(first, first + ninst):
        r = seed(4, i, PURPOSE_LAYERS)
        nx, nz = grids[r.integers(len(grids))]
        h = hs[r.integers(len(hs))]
        nt = int(r.choice(np.arange(1000, 4001, 50)))
        s = int(r.integers(4, 97))
        v_true = layered_model(nz, nx, h, 4, i)
        dt = 1e-3 if 5600.0 * 1e-3 / h <= 0.5 else 5e-4
        g = make_geometry(nz, nx, h, nt, dt, s, rec_stride=2)
        v0 = smooth(v_true, 100.0 / h)
        g = g.replace(vref=float(v0.max()))
        out.append((g, to_m(v_true), to_m(v0)))
    return out


def config5(nshots=96, nt=4000):
    """1024x384 (nx x nz), 12.5 m, 96 shots, 512 receivers; layered model."""
    nz, nx, h = 384, 1024, 12.5
    g = make_geometry(nz, nx, h, nt, 1e-3, nshots, rec_stride=2)
    v_true = layered_model(nz, nx, h, 5, 1000)
    v0 = smooth(v_true, 8.0)
    g = g.replace(vref=float(v0.max()))
    return g, to_m(v_true), to_m(v0)


def learned_instance(instance, nz=128, nx=320, h=12.5, nshots=16, nt=2000):
    """One inversion problem for training or testing the learned direction:
    a layered model with faults (the config-5 family at a reduced size),
    its smoothed starting model, 16 shots and receivers every second cell.
    Training uses instances 0, 1, ...; held-out tests use instances >= 500."""
    g = make_geometry(nz, nx, h, nt, 1e-3, nshots, rec_stride=2)
    v_true = layered_model(nz, nx, h, 5, instance)
    v0 = smooth(v_true, 8.0)
    g = g.replace(vref=float(v0.max()))
    return g, to_m(v_true), to_m(v0)


def uniform_noise(d, snr_db, config, instance=0):
    """Mean-zero uniform noise for the data cube d at the given signal-to-noise
    ratio in dB (10 log10 of mean(d^2) / noise variance), FP32."""
    d = np.asarray(d, np.float64)
    p_sig = float(np.mean(d * d))
    a = np.sqrt(3.0 * p_sig / 10.0 ** (snr_db / 10.0))
    r = seed(config, instance, PURPOSE_NOISE)
    return r.uniform(-a, a, size=d.shape).astype(np.float32)


def small_case(nz=24, nx=28, nb=8, nt=150, nshots=2, nrec=8, h=10.0, dt=1e-3, f0=25.0,
               instance=0):
    """Tiny seeded problem for finite-difference and dot-product checks."""
    r = seed(9, instance, PURPOSE_LAYERS)
    g = make_geometry(nz, nx, h, nt, dt, nshots, rec_stride=max(1, nx // nrec), f0=f0, nb=nb)
    g = g.replace(rec_iz=g.rec_iz[:, :nrec].copy(), rec_ix=g.rec_ix[:, :nrec].copy())
    v = 2000.0 + 600.0 * np.arange(nz)[:, None] / nz + 150.0 * r.standard_normal((nz, nx))
    v = smooth(v, 1.5)
    g = g.replace(vref=float(v.max()))
    return g, to_m(v)
