"""Seeded synthetic X-CT volumes shared by the oracle tests, the GPU tests and
the benchmark.

This module only makes inputs.  It holds none of the reduction method's
arithmetic (no quantisation, threshold, labelling or compaction), so sharing
it does not couple the CPU oracle to the GPU library.

The workloads stand in for the paper's X-CT datasets (Table 1: cylindrical
samples in air, 16-bit slice stacks of up to 42 GB), which are not available
here.  Recipes:

* ``ellipsoids128``: 128^3 float32, N(0.10, 0.02) background, 3 axis-aligned solid
  ellipsoids (semi-axes U[10, 30], level U(0.6, 0.9) + N(0, 0.02)); criterion
  eb = 1e-3 absolute, Otsu, 6-connectivity, keep components of >= 64 voxels.
* ``cylinder1024``: 1024^3 float32 z-axis cylinder, R = 400, air N(0.02, 0.01),
  matrix N(0.5, 0.03), 20 000 pores (r U[2, 12], N(0.05, 0.01)) then 500
  inclusions (r U[3, 8], N(0.95, 0.03)); eb = 1e-4 absolute, Otsu,
  26-connectivity, largest component.
* ``rings2048``: 2048 x 2048 x 1024 uint16 cylinder, R = 633 (30 % of the field
  of view), Gaussian-approximated Poisson counts (mean 12000 inside, 800
  outside) plus 40 ring artefacts of amplitude 200; eb = 1e-4 of the value
  range, Otsu, 26-connectivity, largest component.
* ``batch_volume(j)``: the ellipsoids128 recipe with 1..8 ellipsoids and side
  lengths U{64..512} per axis, eb drawn from {1e-3, 1e-4, 1e-5}.
* ``pixel_section_u8(m)``: an 8-bit pixel section with the make-up of the
  cylinder's region of interest scaled to 0..255 (the normalisation of Sec.
  4.1.2, I_max = 1): matrix N(127.5, 7.65); runs of pore pixels
  N(12.75, 2.55), lengths U{2..20}, over 5.6 % of the section; runs of
  inclusion pixels N(242, 7.65), lengths U{4..14}, over 0.1 %.  The full
  size, 514 688 000 pixels, is the number of span voxels of the 1024^3
  cylinder's extraction.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "roix_synth.c")
_LIB = os.path.join(_HERE, "libroix_synth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library in place (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, u64, dbl, ci = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        vp = ctypes.c_void_p
        lib.synth_ellipsoids_f32.argtypes = [vp, vp, i64, i64, i64, u64, ci, dbl, dbl, dbl, dbl, dbl,
                                             dbl, dbl, ci]
        lib.synth_ellipsoids_f32.restype = ci
        lib.synth_cylinder_f32.argtypes = [vp, vp, i64, i64, i64, u64, dbl, dbl, dbl, dbl, dbl, ci, dbl,
                                           dbl, dbl, dbl, ci, dbl, dbl, dbl, dbl, ci]
        lib.synth_cylinder_f32.restype = ci
        lib.synth_rings_u16.argtypes = [vp, vp, i64, i64, i64, u64, dbl, dbl, dbl, ci, dbl, dbl, ci]
        lib.synth_rings_u16.restype = ci
        lib.synth_rings_u16_planes.argtypes = [vp, vp, i64, i64, i64, i64, u64, dbl, dbl, dbl, ci, dbl, dbl, ci]
        lib.synth_rings_u16_planes.restype = ci
        lib.synth_philox4x32_10.argtypes = [vp, vp, vp]
        lib.synth_philox4x32_10.restype = None
        lib.synth_bernoulli_u8.argtypes = [vp, i64, u64, dbl]
        lib.synth_bernoulli_u8.restype = None
        lib.synth_normal_f32.argtypes = [vp, i64, u64, dbl, dbl, ci]
        lib.synth_normal_f32.restype = None
        _lib = lib
    return _lib


def _threads(n):
    if n is not None:
        return int(n)
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


@dataclass
class Criterion:
    """ROI criterion; mirrors the library's roix_criterion."""
    thr: str = "otsu"            # "otsu" | "fixed"
    fixed_value: float = 0.0
    connectivity: int = 26       # 6 | 26
    keep: str = "largest"        # "largest" | "min_size"
    min_size: int = 1


@dataclass
class Workload:
    name: str
    volume: np.ndarray           # [nz][ny][nx], float32 or uint16
    eb_mode: str                 # "abs" | "rel"
    eb_value: float
    criterion: Criterion
    cls: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def dims(self):
        nz, ny, nx = self.volume.shape
        return nx, ny, nz

    def sha256(self) -> str:
        return hashlib.sha256(np.ascontiguousarray(self.volume).view(np.uint8).data).hexdigest()


def philox4x32_10(ctr, key):
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.synth_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(v) for v in out]


def ellipsoids(nx, ny, nz, seed, n_ell=3, mu_bg=0.10, sd_bg=0.02, ax=(10.0, 30.0), level=(0.6, 0.9),
               sd_obj=0.02, with_cls=False, threads=None):
    lib = _load()
    vol = np.empty((nz, ny, nx), dtype=np.float32)
    cls = np.empty((nz, ny, nx), dtype=np.uint8) if with_cls else None
    rc = lib.synth_ellipsoids_f32(_ptr(vol), _ptr(cls), nx, ny, nz, seed, n_ell, mu_bg, sd_bg, ax[0], ax[1],
                                  level[0], level[1], sd_obj, _threads(threads))
    if rc < 0:
        raise RuntimeError("synth_ellipsoids_f32 failed")
    return vol, cls


def cylinder(nx, ny, nz, seed, R=400.0, air=(0.02, 0.01), matrix=(0.5, 0.03), n_pores=20000,
             pore_r=(2.0, 12.0), pore=(0.05, 0.01), n_incl=500, incl_r=(3.0, 8.0), incl=(0.95, 0.03),
             with_cls=False, threads=None):
    lib = _load()
    vol = np.empty((nz, ny, nx), dtype=np.float32)
    cls = np.empty((nz, ny, nx), dtype=np.uint8) if with_cls else None
    rc = lib.synth_cylinder_f32(_ptr(vol), _ptr(cls), nx, ny, nz, seed, R, air[0], air[1], matrix[0],
                                matrix[1], n_pores, pore_r[0], pore_r[1], pore[0], pore[1], n_incl,
                                incl_r[0], incl_r[1], incl[0], incl[1], _threads(threads))
    if rc < 0:
        raise RuntimeError("synth_cylinder_f32 failed")
    return vol, cls


def rings(nx, ny, nz, seed, R=633.0, lam_in=12000.0, lam_out=800.0, n_rings=40, ring_rmax=1448.0,
          ring_amp=200.0, with_cls=False, threads=None, z0=0, out=None):
    """The rings volume, or its planes [z0, z0 + nz) (slabs cut this way
    assemble into the whole volume exactly); ``out`` may supply the array."""
    lib = _load()
    vol = np.empty((nz, ny, nx), dtype=np.uint16) if out is None else out
    assert vol.shape == (nz, ny, nx) and vol.dtype == np.uint16 and vol.flags.c_contiguous
    cls = np.empty((nz, ny, nx), dtype=np.uint8) if with_cls else None
    rc = lib.synth_rings_u16_planes(_ptr(vol), _ptr(cls), nx, ny, z0, nz, seed, R, lam_in, lam_out, n_rings,
                                    ring_rmax, ring_amp, _threads(threads))
    if rc < 0:
        raise RuntimeError("synth_rings_u16 failed")
    return vol, cls


def bernoulli(shape, seed, p):
    lib = _load()
    out = np.empty(shape, dtype=np.uint8)
    lib.synth_bernoulli_u8(_ptr(out), out.size, seed, p)
    return out


def normal(shape, seed, mu=0.0, sd=1.0, threads=None):
    lib = _load()
    out = np.empty(shape, dtype=np.float32)
    lib.synth_normal_f32(_ptr(out), out.size, seed, mu, sd, _threads(threads))
    return out


def pixel_section_u8(m, seed=4001, threads=None):
    """Seeded 8-bit pixel section of m pixels (recipe in the module notes)."""
    v = normal((m,), seed, 127.5, 7.65, threads)
    rng = np.random.default_rng(seed)
    for frac, lo, hi, mu, sd, s2 in ((0.056, 2, 20, 12.75, 2.55, seed + 1), (0.001, 4, 14, 242.0, 7.65, seed + 2)):
        n_runs = int(frac * m / ((lo + hi) / 2))
        if n_runs == 0 or m <= hi:
            continue
        starts = rng.integers(0, m - hi, n_runs)
        lens = rng.integers(lo, hi + 1, n_runs)
        offs = np.arange(int(lens.sum())) - np.repeat(np.cumsum(lens) - lens, lens)
        idx = np.repeat(starts, lens) + offs
        v[idx] = normal((idx.size,), s2, mu, sd, threads)
    return np.clip(np.rint(v), 0, 255).astype(np.uint8)


PIXEL_SECTION_FULL = 514_688_000


# ------------------------------------------------------------------ workloads

def ellipsoids128(seed=1000, with_cls=False, threads=None) -> Workload:
    vol, cls = ellipsoids(128, 128, 128, seed, n_ell=3, with_cls=with_cls, threads=threads)
    return Workload("128^3 f32 ellipsoids", vol, "abs", 1e-3,
                    Criterion("otsu", 0.0, 6, "min_size", 64), cls)


def cylinder1024(seed=1001, with_cls=False, threads=None, n=1024) -> Workload:
    """The 1024^3 cylinder; ``n`` < 1024 gives the same recipe scaled down
    (radius, pore and inclusion counts scale with the volume)."""
    s = n / 1024.0
    vol, cls = cylinder(n, n, n, seed, R=400.0 * s, n_pores=int(round(20000 * s ** 3)),
                        n_incl=int(round(500 * s ** 3)), with_cls=with_cls, threads=threads)
    return Workload(f"{n}^3 f32 cylinder, pores, inclusions", vol, "abs", 1e-4,
                    Criterion("otsu", 0.0, 26, "largest", 1), cls)


def rings2048(seed=1002, with_cls=False, threads=None, nxy=2048, nz=1024) -> Workload:
    s = nxy / 2048.0
    vol, cls = rings(nxy, nxy, nz, seed, R=633.0 * s, ring_rmax=1448.0 * s, with_cls=with_cls, threads=threads)
    return Workload(f"{nxy}x{nxy}x{nz} u16 cylinder, rings", vol, "rel", 1e-4,
                    Criterion("otsu", 0.0, 26, "largest", 1), cls)


def batch_volume(j, seed_base=2000, with_cls=False, threads=None, side=(64, 512)) -> Workload:
    """Volume j of the 64-volume batch: sides U{64..512} per axis, 1..8
    ellipsoids, eb from {1e-3, 1e-4, 1e-5}; all draws from Philox with this
    volume's seed."""
    seed = seed_base + j
    # parameter stream distinct from the generator's own streams
    r = philox4x32_10([j, 0, 0, 0], [seed & 0xFFFFFFFF, 0x5EED])
    lo, hi = side
    nx = lo + r[0] % (hi - lo + 1)
    ny = lo + r[1] % (hi - lo + 1)
    nz = lo + r[2] % (hi - lo + 1)
    n_ell = 1 + r[3] % 8
    eb = (1e-3, 1e-4, 1e-5)[philox4x32_10([j, 1, 0, 0], [seed & 0xFFFFFFFF, 0x5EED])[0] % 3]
    vol, cls = ellipsoids(nx, ny, nz, seed, n_ell=n_ell, with_cls=with_cls, threads=threads)
    return Workload(f"batch[{j}]: {nx}x{ny}x{nz} f32, {n_ell} ellipsoids", vol, "abs", eb,
                    Criterion("otsu", 0.0, 6, "min_size", 64), cls, {"n_ell": n_ell})


def served_calibration(seed=3999, nxy=2048, nz=8, threads=None) -> np.ndarray:
    """The calibration volume of the served streams (rings recipe): its value
    range sets the streams' absolute bound."""
    vol, _ = rings(nxy, nxy, nz, seed, threads=threads)
    return vol


def served_stream(k, nz=256, nxy=2048, seed_base=3001, threads=None) -> np.ndarray:
    """Stream k of the served trace: a uint16 rings volume (cylinder, Poisson
    noise, ring artefacts) of nxy x nxy x nz, sent in 32-plane slabs."""
    s = nxy / 2048.0
    vol, _ = rings(nxy, nxy, nz, seed_base + k, R=633.0 * s, ring_rmax=1448.0 * s, threads=threads)
    return vol


def served_slab(k, z0, nz=32, nxy=2048, seed_base=3001, threads=None, out=None) -> np.ndarray:
    """Planes [z0, z0 + nz) of served stream k (generated alone, so a trace
    need not hold whole streams in memory)."""
    s = nxy / 2048.0
    vol, _ = rings(nxy, nxy, nz, seed_base + k, R=633.0 * s, ring_rmax=1448.0 * s, threads=threads, z0=z0, out=out)
    return vol


def served_cube(k, seed_base=3100, side=(128, 512), threads=None) -> Workload:
    """Cube k of the served trace: a float32 ellipsoid volume with sides drawn
    from U{side} (the small-volume recipe), sent whole."""
    seed = seed_base + k
    r = philox4x32_10([k, 2, 0, 0], [seed & 0xFFFFFFFF, 0x5EED])
    lo, hi = side
    n = lo + r[0] % (hi - lo + 1)
    n_ell = 1 + r[1] % 8
    vol, _ = ellipsoids(n, n, n, seed, n_ell=n_ell, threads=threads)
    return Workload(f"served cube {k}: {n}^3 f32, {n_ell} ellipsoids", vol, "abs", 1e-3,
                    Criterion("otsu", 0.0, 6, "min_size", 64), None)
