"""Pins of the CPU oracle against things other than itself.

Each test checks one oracle function against a closed form, an invariant,
an exact-arithmetic evaluation, an independent library or brute force, or a
hand-derived worked example -- chosen so that a plausible slip in the oracle
(a dropped term, a wrong sign or index, an off-by-one span end, a transposed
axis, the wrong rounding rule) fails at least one of them.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ inputs

def test_philox_known_answers():
    # Known-answer vectors of Philox4x32-10 (Salmon et al., SC'11, Random123 KAT).
    assert synth.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert synth.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6,
                                                                       0x6D5451FD]
    assert synth.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == [
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_generator_thread_invariance():
    a = synth.cylinder1024(n=96, threads=1).volume
    b = synth.cylinder1024(n=96, threads=4).volume
    assert a.tobytes() == b.tobytes()


# ------------------------------------------------------------------- range

def test_range_matches_numpy_and_signed_zero():
    w = synth.ellipsoids128()
    st, lo, hi = oracle.value_range(w.volume)
    assert st == oracle.OK and lo == w.volume.min() and hi == w.volume.max()
    v = np.array([0.0, -0.0, 0.0], np.float32)
    st, lo, hi = oracle.value_range(v)
    assert np.signbit(lo) and not np.signbit(hi)          # IEEE total order: -0 < +0
    u = np.array([7, 0, 65535, 3], np.uint16)
    assert oracle.value_range(u)[1:] == (0.0, 65535.0)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_range_rejects_non_finite(bad):
    v = np.ones(100, np.float32)
    v[57] = bad
    assert oracle.value_range(v)[0] == oracle.EINVAL


# ----------------------------------------------------------------- resolve

def test_eb_rounds_down_to_fp32():
    # float32(1e-3) rounds up, so the fp32 bound must step down; float32(1e-4) rounds down.
    p = oracle.resolve(0.0, 1.0, "abs", 1e-3)
    assert p.status == 0 and np.float32(p.eb32) == np.nextafter(np.float32(1e-3), np.float32(0))
    assert float(np.float32(p.eb32)) <= 1e-3
    p = oracle.resolve(0.0, 1.0, "abs", 1e-4)
    assert np.float32(p.eb32) == np.float32(1e-4) and float(np.float32(1e-4)) <= 1e-4
    # w = 2 eb exactly, r = fl(1/w) (correctly rounded; binary64 quotient rounded once more is
    # the same value since 53 >= 2*24+2)
    assert np.float32(p.w) == np.float32(2) * np.float32(p.eb32)
    assert np.float32(p.r) == np.float32(1.0 / float(np.float32(p.w)))


def test_eb_relative_and_errors():
    p = oracle.resolve(100.0, 65000.0, "rel", 1e-4)
    assert np.float32(p.eb32) <= 1e-4 * (65000.0 - 100.0)
    assert oracle.resolve(5.0, 5.0, "rel", 1e-4).status == oracle.EINVAL       # constant volume
    assert oracle.resolve(0.0, 1.0, "abs", 0.0).status == oracle.EINVAL
    assert oracle.resolve(0.0, 1.0, "abs", -1.0).status == oracle.EINVAL
    assert oracle.resolve(0.0, 1.0, "abs", float("nan")).status == oracle.EINVAL
    assert oracle.resolve(0.0, 1.0, "abs", 1e-45).status == oracle.EINVAL      # not a normal float
    assert oracle.resolve(0.0, 1e4, "abs", 1e-6).status == oracle.ERANGE       # |x r| > 2^24
    assert oracle.resolve(-1e4, 0.0, "abs", 1e-6).status == oracle.ERANGE


def test_width_selection():
    assert oracle.resolve(0.0, 254 * 2 ** -9, "abs", 2 ** -10).width_bits == 8     # K = 255
    assert oracle.resolve(0.0, 255 * 2 ** -9, "abs", 2 ** -10).width_bits == 16    # K = 256
    p = oracle.resolve(0.0, 65534 * 2 ** -9, "abs", 2 ** -10)
    assert (p.K, p.width_bits, p.esc) == (65535, 16, 65535)
    p = oracle.resolve(0.0, 65535 * 2 ** -9, "abs", 2 ** -10)
    assert (p.K, p.width_bits, p.esc) == (65536, 32, 0xFFFFFFFF)


# ---------------------------------------------------------------- quantise

def test_codes_closed_form_on_grid_points():
    # eb = 2^-10: w = 2^-9 and r = 512 are exact, so x = k w gives q = k and
    # x = (k + 1/2) w is an exact tie that rounds to the even neighbour.
    k = np.arange(-3000, 3000, dtype=np.int64)
    x = (k.astype(np.float64) / 512.0).astype(np.float32)
    p = oracle.resolve(float(x.min()), float(x.max()), "abs", 2.0 ** -10)
    st, q, bits, nout = oracle.quantize(x, p)
    assert st == 0 and nout == 0 and np.array_equal(q, k)
    xt = ((k.astype(np.float64) + 0.5) / 512.0).astype(np.float32)
    p = oracle.resolve(float(xt.min()), float(xt.max()), "abs", 2.0 ** -10)
    st, q, bits, nout = oracle.quantize(xt, p)
    even = np.where(k % 2 == 0, k, k + 1)
    assert np.array_equal(q, even)


def test_codes_bound_and_exact_rounding_cross_check():
    w = synth.ellipsoids128()
    x = w.volume.ravel()
    _, lo, hi = oracle.value_range(x)
    p = oracle.resolve(lo, hi, "abs", 1e-3)
    st, q, bits, nout = oracle.quantize(x, p)
    # invariant: the decoded value fl(q w) is within eb of x for every non-outlier voxel; the
    # difference of two floats is taken exactly in binary64
    wv = float(np.float32(p.w))
    xh = q.astype(np.float32) * np.float32(p.w)
    err = np.abs(x.astype(np.float64) - xh.astype(np.float64))
    outl = np.unpackbits(bits.view(np.uint8), bitorder="little")[: x.size].astype(bool)
    assert nout == outl.sum()
    assert float(np.float32(p.eb32)) <= 1e-3
    assert np.all(err[~outl] <= float(np.float32(p.eb32)))
    # exact arithmetic: q equals round-half-even(x / w) except within the two fp32 roundings of a half
    t = x.astype(np.float64) / wv                       # relative error 2^-53
    qe = np.rint(t)
    dist = np.abs(np.abs(t - np.floor(t)) - 0.5)
    far = dist > 2.0 ** -21 * np.maximum(np.abs(t), 1.0)
    assert far.mean() > 0.99
    assert np.array_equal(q[far], qe[far].astype(np.int32))
    # code domain: q is monotone in x, so the extremes give qmin/qmax
    assert q.min() == p.qmin and q.max() == p.qmax


def test_outliers_exist_and_are_the_only_bound_failures():
    # a dense uniform sweep at a small bound produces fp32 bound failures (escapes)
    x = np.linspace(0.0, 1.0, 2_000_001, dtype=np.float32)
    p = oracle.resolve(0.0, 1.0, "abs", 1e-5)
    st, q, bits, nout = oracle.quantize(x, p)
    outl = np.unpackbits(bits.view(np.uint8), bitorder="little")[: x.size].astype(bool)
    xh = (q.astype(np.float32) * np.float32(p.w)).astype(np.float32)
    fail = ~(np.abs(x - xh) <= np.float32(p.eb32))
    assert nout > 0 and np.array_equal(outl, fail)


# --------------------------------------------------------------- histogram

def test_histogram_special_cases():
    # K = 256: bin = q - qmin (identity);  K = 512: bin = (q - qmin) // 2
    for K in (256, 512, 1000):
        k = np.arange(K, dtype=np.int64)
        x = (k / 512.0).astype(np.float32)
        p = oracle.resolve(0.0, float(x.max()), "abs", 2.0 ** -10)
        assert p.K == K
        _, q, _, _ = oracle.quantize(x, p)
        h = oracle.histogram(q, p)
        assert h.sum() == K
        if K == 256:
            assert np.all(h == 1)
        elif K == 512:
            assert np.all(h == 2)
        else:
            # equal-width bins over the code range: every bin holds floor or ceil of K/256 codes,
            # and bin t starts at the first u with 256 u >= t K
            assert set(np.unique(h)) <= {K // 256, K // 256 + 1}
            starts = np.concatenate([[0], np.cumsum(h)[:-1]])
            for t in range(256):
                u = int(starts[t])
                assert 256 * u >= t * K and (u == 0 or 256 * (u - 1) < t * K)


# -------------------------------------------------------------------- Otsu

def _otsu_exact(h):
    """Exact rational between-class criterion for every split; first maximum."""
    h = [int(v) for v in h]
    NT = sum(h)
    ST = sum(i * v for i, v in enumerate(h))
    best, arg, vals = None, 255, []
    W0 = S0 = 0
    for t in range(255):
        W0 += h[t]
        S0 += t * h[t]
        W1 = NT - W0
        if W0 == 0 or W1 == 0:
            vals.append(None)
            continue
        # sigma_B^2 * NT^2 = (S0 W1 - S1 W0)^2 / (W0 W1)
        s = Fraction((S0 * W1 - (ST - S0) * W0) ** 2, W0 * W1)
        vals.append(s)
        if best is None or s > best:
            best, arg = s, t
    return arg, vals


@pytest.mark.parametrize("seed", range(40))
def test_otsu_brute_force_random(seed):
    rng = np.random.default_rng(seed)
    h = np.zeros(256, np.uint64)
    kind = seed % 4
    if kind == 0:
        h[:] = rng.integers(0, 1000, 256)
    elif kind == 1:                       # bimodal
        for c, s, n in ((60, 10, 50000), (190, 15, 30000)):
            b = np.clip(np.rint(rng.normal(c, s, n)), 0, 255).astype(int)
            h += np.bincount(b, minlength=256).astype(np.uint64)
    elif kind == 2:                       # sparse
        idx = rng.choice(256, 5, replace=False)
        h[idx] = rng.integers(1, 10 ** 9, 5)
    else:                                 # large counts
        h[:] = rng.integers(0, 2 ** 30, 256)
    t, flags = oracle.otsu(h)
    te, vals = _otsu_exact(h)
    finite = [v for v in vals if v is not None]
    top = sorted(finite, reverse=True)[:2]
    # no near-tie between the two best splits (so double rounding cannot flip the argmax)
    if len(top) == 2 and top[0] != top[1]:
        assert float((top[0] - top[1]) / top[0]) > 1e-12
    assert t == te and flags == 0


def test_otsu_closed_forms():
    h = np.zeros(256, np.uint64)
    h[37], h[201] = 1000, 5
    assert oracle.otsu(h) == (37, 0)          # two spikes i<j: every t in [i, j) ties, first wins
    h = np.zeros(256, np.uint64)
    h[100] = 77
    assert oracle.otsu(h) == (255, oracle.FLAG_DEGENERATE)   # one class only
    assert oracle.otsu(np.zeros(256, np.uint64)) == (255, oracle.FLAG_DEGENERATE)


def _multi_exact(h, K):
    """Multi-level Otsu by exact rationals: every partition of the non-empty
    bins into K contiguous non-empty classes, scored by sum_k S_k^2 / W_k
    (the between-class variance up to a positive factor and a constant).
    Returns the best score, the runner-up score and the lexicographically
    smallest threshold tuple of the best partition (a cut after non-empty bin
    p is the threshold p, the smallest bin index that realises it)."""
    from itertools import combinations
    pos = [i for i in range(256) if h[i]]
    scored = []
    for cuts in combinations(range(len(pos) - 1), K - 1):
        bounds = [-1] + list(cuts) + [len(pos) - 1]
        score = Fraction(0)
        for a, b in zip(bounds[:-1], bounds[1:]):
            W = sum(int(h[pos[j]]) for j in range(a + 1, b + 1))
            S = sum(pos[j] * int(h[pos[j]]) for j in range(a + 1, b + 1))
            score += Fraction(S * S, W)
        scored.append((score, tuple(pos[c] for c in cuts)))
    scored.sort(key=lambda e: (-e[0], e[1]))
    runner = scored[1][0] if len(scored) > 1 else None
    return scored[0][0], runner, scored[0][1]


@pytest.mark.parametrize("seed", range(24))
def test_multi_otsu_exact_partitions(seed):
    # the oracle's binary64 search against an exact search over partitions
    rng = np.random.default_rng(9000 + seed)
    K = 3 if seed % 2 == 0 else 4
    m = int(rng.integers(K, 11))
    h = np.zeros(256, np.uint64)
    idx = np.sort(rng.choice(256, m, replace=False))
    h[idx] = rng.integers(1, 10 ** (3 + seed % 6), m)
    best, runner, tup = _multi_exact(h, K)
    if runner is not None and best != runner:
        assert float((best - runner) / best) > 1e-12  # no near-tie the rounding could flip
    got, flags = oracle.multi_otsu(h, K)
    assert flags == 0 and got == tup, (K, idx.tolist(), got, tup)


def test_multi_otsu_closed_forms():
    # exactly K non-empty bins: the only valid tuple cuts after each but the last
    h = np.zeros(256, np.uint64)
    h[[3, 90, 250]] = [5, 1, 2]
    assert oracle.multi_otsu(h, 3) == ((3, 90), 0)
    h[7] = 4
    assert oracle.multi_otsu(h, 4) == ((3, 7, 90), 0)
    # fewer non-empty bins than classes: no valid tuple, empty mask
    h = np.zeros(256, np.uint64)
    h[[10, 20]] = 6
    assert oracle.multi_otsu(h, 3) == ((255, 255), oracle.FLAG_DEGENERATE)
    assert oracle.multi_otsu(np.zeros(256, np.uint64), 4) == ((255, 255, 255), oracle.FLAG_DEGENERATE)
    # two well-separated groups of bins per threshold: the thresholds fall in the gaps
    h = np.zeros(256, np.uint64)
    h[20:30] = 1000
    h[120:130] = 1000
    h[220:230] = 1000
    (t1, t2), _ = oracle.multi_otsu(h, 3)
    assert 29 <= t1 < 120 and 129 <= t2 < 220


def test_multi_otsu_three_materials():
    # background, matrix and inclusions of distinct intensities: three-class
    # Otsu keeps everything above the background; four classes split no material
    rng = np.random.default_rng(77)
    vol = np.full((12, 24, 32), 0.1, np.float64) + rng.normal(0, 0.01, (12, 24, 32))
    vol[2:10, 4:20, 6:26] = 0.5 + rng.normal(0, 0.01, (8, 16, 20))
    vol[4:8, 8:14, 10:16] = 0.9 + rng.normal(0, 0.01, (4, 6, 6))
    vol = vol.astype(np.float32)
    fg = int(((vol > 0.3)).sum())
    r = oracle.fused(vol, "abs", 1e-3, "multi3", 0.0, 6, "min_size", 1)
    assert r["status"] == 0 and r["info"].n_classes == 3
    assert r["info"].n_mask == fg
    t = list(r["info"].thresholds)
    assert t[0] < t[1] and t[2] == -1 and r["info"].otsu_bin == t[0]
    r4 = oracle.fused(vol, "abs", 1e-3, "multi4", 0.0, 6, "min_size", 1)
    assert r4["status"] == 0 and r4["info"].n_classes == 4 and r4["info"].thresholds[0] < r4["info"].thresholds[1] < r4["info"].thresholds[2]


def test_threshold_mask_equivalence():
    # q >= q_thr  <=>  bin(q) > t*  for every code of the range (Otsu); q > q(T) for FIXED
    for K in (7, 255, 256, 1000, 65537):
        x = (np.arange(K) / 512.0).astype(np.float32)
        p = oracle.resolve(0.0, float(x.max()), "abs", 2.0 ** -10)
        u = np.arange(K, dtype=np.int64)
        b = (u * 256) // K                               # bins by their integer definition
        for t in (0, 1, 100, 254, 255):
            qt = oracle.q_thr_otsu(t, p)
            assert np.array_equal(u + p.qmin >= qt, b > t)
    p = oracle.resolve(0.0, 1.0, "abs", 2.0 ** -10)
    assert oracle.q_thr_fixed(100 / 512, p) == 101
    assert oracle.q_thr_fixed(-5.0, p) == p.qmin           # below the range: everything is object
    assert oracle.q_thr_fixed(99.0, p) == p.qmax + 1       # above the range: nothing is object


# ---------------------------------------------------------------- labelling

def _scipy_canonical(mask, conn):
    st = ndi.generate_binary_structure(3, 1 if conn == 6 else 3)
    lab, n = ndi.label(mask, structure=st)
    flat = lab.ravel()
    out = np.full(flat.shape, -1, np.int64)
    idx = np.flatnonzero(flat)
    # canonical label = smallest linear index of the component
    first = np.full(n + 1, np.iinfo(np.int64).max, np.int64)
    np.minimum.at(first, flat[idx], idx)
    out[idx] = first[flat[idx]]
    return out.reshape(mask.shape), n


def _patterns():
    yield "checker", (np.indices((6, 7, 8)).sum(0) % 2).astype(np.uint8)
    s = np.zeros((5, 9, 9), np.uint8)                 # snake: one long chain with many turns
    s[:, ::2, :] = 1
    for y in range(1, 9, 2):
        s[:, y, 8 if (y // 2) % 2 == 0 else 0] = 1
    yield "snake", s
    h = np.zeros((16, 12, 12), np.uint8)              # helix (diagonal steps, 26- vs 6-connectivity)
    for z in range(16):
        a = z * np.pi / 4
        h[z, int(round(6 + 4 * np.sin(a))), int(round(6 + 4 * np.cos(a)))] = 1
    yield "helix", h
    c = np.zeros((4, 8, 16), np.uint8)                # comb: teeth joined by a spine
    c[:, :, ::2] = 1
    c[:, 0, :] = 1
    yield "comb", c
    d = np.zeros((3, 3, 3), np.uint8)                 # diagonal corner contacts only
    d[0, 0, 0] = d[1, 1, 1] = d[2, 2, 2] = 1
    yield "corners", d


@pytest.mark.parametrize("conn", [6, 26])
def test_label_vs_scipy_random(conn):
    rng = np.random.default_rng(conn)
    for trial in range(60):
        shape = tuple(int(s) for s in rng.integers(1, 13, 3))
        p = float(rng.uniform(0.05, 0.95))
        mask = synth.bernoulli(shape, 7000 + trial, p)
        st, lab, keep, comps = oracle.label(mask, conn, keep="min_size", min_size=1)
        ref, n = _scipy_canonical(mask, conn)
        assert st == 0 and np.array_equal(lab, ref) and len(comps) == n
        assert keep.sum() == mask.sum()


@pytest.mark.parametrize("conn", [6, 26])
def test_label_adversarial_patterns(conn):
    for name, mask in _patterns():
        st, lab, keep, comps = oracle.label(mask, conn, keep="min_size", min_size=1)
        ref, n = _scipy_canonical(mask, conn)
        assert np.array_equal(lab, ref), name
        # sizes and half-open boxes against numpy
        for c in comps:
            zz, yy, xx = np.nonzero(lab == c["label"])
            assert c["size"] == len(xx)
            assert (c["x0"], c["x1"], c["y0"], c["y1"], c["z0"], c["z1"]) == (
                xx.min(), xx.max() + 1, yy.min(), yy.max() + 1, zz.min(), zz.max() + 1)
    assert len(oracle.label(dict(_patterns())["corners"], 6)[3]) == 3
    assert len(oracle.label(dict(_patterns())["corners"], 26)[3]) == 1


def test_keep_rules():
    m = np.zeros((1, 5, 12), np.uint8)
    m[0, 0, 0:3] = 1      # size 3, label 0
    m[0, 2, 5:8] = 1      # size 3, label 29 (tie -> smaller label wins)
    m[0, 4, 0:2] = 1      # size 2
    st, lab, keep, comps = oracle.label(m, 26, keep="largest")
    assert [c["kept"] for c in comps] == [1, 0, 0]
    assert keep.sum() == 3 and keep[0, 0, 0:3].all()
    st, lab, keep, comps = oracle.label(m, 26, keep="min_size", min_size=3)
    assert [c["kept"] for c in comps] == [1, 1, 0]
    st, lab, keep, comps = oracle.label(m, 26, keep="min_size", min_size=1, comps_cap=2)
    assert st == oracle.ETRUNC and len(comps) == 2


# --------------------------------------------------------- rows and stream

def test_rows_against_numpy():
    rng = np.random.default_rng(3)
    keep = (rng.random((4, 9, 33)) < 0.1).astype(np.uint8)
    rt = oracle.rows(keep)
    exp = []
    for z in range(4):
        for y in range(9):
            xs = np.flatnonzero(keep[z, y])
            if len(xs):
                exp.append((z, y, xs[0], xs[-1] + 1))
    assert [(r["z"], r["y"], r["xs"], r["xe"]) for r in rt] == exp


def test_hand_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "hand_rows.json")))
    k = np.array(g["k"], np.float64).reshape(g["shape_zyx"])
    vol = (k / 512.0).astype(np.float32)
    e = g["expected"]
    T = g["fixed_T_k"] / 512.0
    for keep, key in (("largest", "largest"), ("min_size", "min_size_1")):
        for conn in (6, 26):
            r = oracle.fused(vol, "abs", g["eb"], thr="fixed", fixed_value=T, connectivity=conn, keep=keep,
                             min_size=1)
            p = r["params"]
            assert r["status"] == 0
            assert (p.qmin, p.qmax, p.K, p.width_bits) == (e["qmin"], e["qmax"], e["K"], e["width_bits"])
            got = [{"label": int(c["label"]), "size": int(c["size"]),
                    "bbox": [int(c[f]) for f in ("x0", "x1", "y0", "y1", "z0", "z1")]} for c in r["comps"]]
            assert got == e["components"]
            rows = [[int(x) for x in row] for row in r["rows"].tolist()]
            assert rows == e[key]["rows"]
            assert r["stream"].tolist() == e[key]["stream"]


def test_decode_round_trip_and_span_invariants():
    w = synth.ellipsoids128(with_cls=True)
    c = w.criterion
    r = oracle.fused(w.volume, w.eb_mode, w.eb_value, c.thr, 0.0, c.connectivity, c.keep, c.min_size)
    p, info = r["params"], r["info"]
    rt = r["rows"]
    assert info.n_codes == int((rt["xe"].astype(np.int64) - rt["xs"]).sum())
    assert np.all(np.diff(rt["code_off"].astype(np.int64)) == (rt["xe"] - rt["xs"])[:-1])
    st, out = oracle.decode(rt, r["stream"], r["outliers"], p, w.volume.shape, background=np.nan)
    assert st == 0
    span = ~np.isnan(out)
    assert span.sum() == info.n_codes
    err = np.abs(out[span].astype(np.float64) - w.volume[span].astype(np.float64))
    assert err.max() <= float(np.float32(p.eb32))
    # span endpoints are kept voxels: compare with an independent labelling of the mask
    mask = w.cls > 0
    ref, n = _scipy_canonical(mask.astype(np.uint8), 6)
    for row in rt[:: max(1, len(rt) // 200)]:
        assert ref[row["z"], row["y"], row["xs"]] >= 0 and ref[row["z"], row["y"], row["xe"] - 1] >= 0


def test_etrunc_reports_full_counts():
    w = synth.ellipsoids128()
    c = w.criterion
    full = oracle.fused(w.volume, w.eb_mode, w.eb_value, c.thr, 0.0, c.connectivity, c.keep, c.min_size)
    small = oracle.fused(w.volume, w.eb_mode, w.eb_value, c.thr, 0.0, c.connectivity, c.keep, c.min_size,
                         rows_cap=10, stream_cap_bytes=100, outliers_cap=0)
    assert small["status"] == oracle.ETRUNC
    assert small["info"].n_rows == full["info"].n_rows and small["info"].n_codes == full["info"].n_codes
    assert small["stream"].tolist() == full["stream"][:100].tolist()
    cut = oracle.fused(w.volume, w.eb_mode, w.eb_value, c.thr, 0.0, c.connectivity, c.keep, c.min_size,
                       comps_cap=2)
    assert cut["status"] == oracle.ETRUNC and cut["info"].n_components == full["info"].n_components


# ------------------------------------------------------------- ground truth

def _dsc(a, b):
    a, b = a.astype(bool), b.astype(bool)
    return 2.0 * (a & b).sum() / (a.sum() + b.sum())


def test_ground_truth_ellipsoids128():
    w = synth.ellipsoids128(with_cls=True)
    c = w.criterion
    r = oracle.fused(w.volume, w.eb_mode, w.eb_value, c.thr, 0.0, c.connectivity, c.keep, c.min_size)
    info = r["info"]
    truth = w.cls > 0
    # the classes are >= 7 sd apart, so the mask is exactly the analytic object set
    assert info.n_mask == truth.sum()
    _, n = _scipy_canonical(truth.astype(np.uint8), 6)
    assert info.n_components == n and info.n_kept == n
    assert _dsc(truth, truth) == 1.0


def test_ground_truth_cylinder_spans():
    w = synth.cylinder1024(n=160, with_cls=True)
    c = w.criterion
    r = oracle.fused(w.volume, w.eb_mode, w.eb_value, c.thr, 0.0, c.connectivity, c.keep, c.min_size)
    info = r["info"]
    fg = (w.cls == 1) | (w.cls == 3)
    assert info.n_mask == fg.sum()
    st, lab, keep, comps = oracle.label(fg.astype(np.uint8), 26, keep="largest")
    big = comps[np.argmax(comps["size"])]
    assert info.n_kept_voxels == big["size"]
    # rows: the chord of the cylinder wall (pores stay >= 1 voxel inside it)
    exp = []
    for z in range(fg.shape[0]):
        for y in range(fg.shape[1]):
            xs = np.flatnonzero(keep[z, y])
            if len(xs):
                exp.append((z, y, xs[0], xs[-1] + 1))
    got = [(a["z"], a["y"], a["xs"], a["xe"]) for a in r["rows"]]
    assert got == exp


def test_ground_truth_rings_u16():
    w = synth.rings2048(nxy=256, nz=8, with_cls=True)
    c = w.criterion
    r = oracle.fused(w.volume, w.eb_mode, w.eb_value, c.thr, 0.0, c.connectivity, c.keep, c.min_size)
    info = r["info"]
    assert r["status"] == 0 and info.n_mask == (w.cls == 1).sum() and info.n_components == 1
    st, out = oracle.decode(r["rows"], r["stream"], r["outliers"], r["params"], w.volume.shape, np.nan)
    span = ~np.isnan(out)
    assert np.abs(out[span] - w.volume[span].astype(np.float32)).max() <= np.float32(r["params"].eb32)


def _dyadic_object_and_background(shape, seed, planes):
    # object values on a 2^-12 grid in [0, 1), background on a 2^-8 grid in
    # [0, 2): every sum is exact in float32 (at most 14 significant bits)
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    obj = (rng.integers(0, 4096, shape) / 4096.0).astype(np.float32)
    bg = (rng.integers(0, 512, (planes, ny, nx)) / 256.0).astype(np.float32)
    return obj, bg, (obj + bg).astype(np.float32)


def test_background_subtraction_recovers_the_object():
    # Sec. 4.1.1: M = I - B; with I = O + B exact, M is O to the bit, and
    # adding B back (the reverse process) gives I to the bit
    for planes in (1, 5):
        obj, bg, img = _dyadic_object_and_background((5, 7, 9), 90 + planes, planes)
        st, m = oracle.background(img, bg)
        assert st == oracle.OK and m.view(np.uint32).tobytes() == obj.view(np.uint32).tobytes()
        st, back = oracle.background(m, bg, "add")
        assert st == oracle.OK and back.view(np.uint32).tobytes() == img.view(np.uint32).tobytes()
    # one plane for every z == the same plane repeated as a volume
    obj, bg, img = _dyadic_object_and_background((4, 6, 10), 95, 1)
    assert np.array_equal(oracle.background(img, bg)[1], oracle.background(img, np.repeat(bg, 4, axis=0))[1])
    # uint16 input converts exactly: subtracting its own float values gives zeros
    u = np.random.default_rng(96).integers(0, 65536, (3, 4, 5)).astype(np.uint16)
    st, m = oracle.background(u, u.astype(np.float32))
    assert st == oracle.OK and not m.any()
    st, m = oracle.background(u, np.zeros((1, 4, 5), np.float32))
    assert np.array_equal(m, u.astype(np.float32))
    # the reference must be one plane or one per z
    assert oracle.background(u, np.zeros((2, 4, 5), np.float32))[0] == oracle.EINVAL


def test_background_subtraction_isolates_the_object():
    # a strong background field hides the object from the threshold; after
    # subtraction the path sees exactly the object volume
    nz, ny, nx = 8, 32, 48
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    obj = np.where((x - 24) ** 2 + (y - 16) ** 2 + 4 * (z - 4) ** 2 < 81, 0.5, 0.0)
    obj = (np.round(obj * 4096) / 4096).astype(np.float32)
    ramp = np.round(2.0 * np.arange(nx) / nx * 256) / 256          # 0 .. 2 across x, on a 2^-8 grid
    bg = np.broadcast_to(ramp, (1, ny, nx)).astype(np.float32)
    img = (obj + bg).astype(np.float32)
    st, m = oracle.background(img, bg)
    assert st == oracle.OK and np.array_equal(m, obj)
    ref = oracle.fused(obj, "abs", 1e-3, "otsu", 0.0, 26, "largest", 1)
    sub = oracle.fused(m, "abs", 1e-3, "otsu", 0.0, 26, "largest", 1)
    raw = oracle.fused(img, "abs", 1e-3, "otsu", 0.0, 26, "largest", 1)
    n_obj = int((obj > 0).sum())
    assert ref["info"].n_kept_voxels == n_obj and sub["info"].n_kept_voxels == n_obj
    assert sub["rows"].tobytes() == ref["rows"].tobytes() and sub["stream"].tobytes() == ref["stream"].tobytes()
    assert raw["info"].n_kept_voxels != n_obj  # without the subtraction the ramp decides the mask


def _min_groups(d, K):
    # fewest contiguous groups with max - min <= K, by dynamic programming
    # over every split (independent of the greedy scan)
    n = len(d)
    best = [0] + [n + 1] * n
    for j in range(1, n + 1):
        lo = hi = int(d[j - 1])
        for i in range(j - 1, -1, -1):
            lo, hi = min(lo, int(d[i])), max(hi, int(d[i]))
            if hi - lo > K:
                break
            best[j] = min(best[j], best[i] + 1)
    return best[n]


def test_abs_quantize_hand_examples():
    g = json.load(open(os.path.join(GOLDEN, "hand_abs_quantize.json")))
    for c in g["cases"]:
        st, q, n = oracle.abs_quantize(np.array(c["D"], np.uint8), c["E"])
        assert st == oracle.OK and q.tolist() == c["Q"] and n == c["groups"], c


def test_abs_quantize_bound_and_optimal_group_count():
    # Sec. 4.2.3: |Q - D| <= E for every pixel; the greedy growth gives the
    # fewest groups (checked against an exhaustive dynamic programme); Q
    # changes value only between groups
    rng = np.random.default_rng(97)
    for trial in range(300):
        n = int(rng.integers(1, 60))
        kind = trial % 3
        if kind == 0:
            d = rng.integers(0, 256, n)
        elif kind == 1:
            d = np.clip(np.round(128 + np.cumsum(rng.normal(0, 2, n))), 0, 255)
        else:
            d = np.clip(np.round(rng.normal(120, 6, n)), 0, 255)
        d = d.astype(np.uint8)
        e = float(rng.choice([0.0, 0.3, 1.0, 1.7, 2.0, 3.0, 5.5, 20.0]))
        st, q, groups = oracle.abs_quantize(d, e)
        ei = int(np.floor(e))
        assert st == oracle.OK
        assert np.all(np.abs(q.astype(int) - d.astype(int)) <= ei)
        assert groups == _min_groups(d, 2 * ei)
        assert int((np.diff(q.astype(int)) != 0).sum()) <= groups - 1


def test_abs_quantize_closed_forms():
    # constant pixels: one group, Q = D
    st, q, n = oracle.abs_quantize(np.full(50, 77, np.uint8), 3)
    assert n == 1 and np.all(q == 77)
    # E < 1: groups are the runs of equal pixels and Q = D
    d = np.array([5, 5, 6, 6, 6, 5, 200, 200, 0], np.uint8)
    st, q, n = oracle.abs_quantize(d, 0.9)
    assert np.array_equal(q, d) and n == 5
    # ramp 0, 1, 2, ...: groups of 2E + 1 pixels written at their centre
    for e in (1, 2, 4):
        d = np.arange(200, dtype=np.uint8)
        st, q, n = oracle.abs_quantize(d, e)
        L = 2 * e + 1
        assert n == -(-200 // L)
        full = (200 // L) * L
        assert np.array_equal(q[:full], (np.arange(full) // L) * L + e)
        if full < 200:  # the last, shorter group: floor of its midpoint
            assert np.all(q[full:] == (full + 199) // 2)
    # a tolerance covering the whole 8-bit range: one group at (min + max) / 2
    d = np.array([0, 255, 17, 3], np.uint8)
    st, q, n = oracle.abs_quantize(d, 128)
    assert n == 1 and np.all(q == 127)
    # empty input and a negative tolerance
    assert oracle.abs_quantize(np.zeros(0, np.uint8), 1)[2] == 0
    assert oracle.abs_quantize(d, -1.0)[0] == oracle.EINVAL


def _huffman_cost(counts):
    # optimal total code length of a prefix code: the sum of the merged
    # weights of any Huffman construction (heap order is irrelevant to it)
    import heapq
    h = [int(c) for c in counts if c > 0]
    if len(h) <= 1:
        return sum(h)
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def _canonical_decode(lengths, block_off, payload, n):
    # decoder written from the format definition: canonical codes by
    # (length, byte), most significant bit first, blocks of 4096 bytes on
    # fresh 32-bit words
    items = sorted((int(l), s) for s, l in enumerate(lengths) if l)
    table, code, prev = {}, 0, items[0][0] if items else 0
    for i, (l, s) in enumerate(items):
        if i:
            code = (code + 1) << (l - prev)
        prev = l
        table[(l, code)] = s
    out = []
    for b in range(len(block_off) - 1):
        bits = "".join(f"{int(w):032b}" for w in payload[int(block_off[b]): int(block_off[b + 1])])
        p = 0
        for _ in range(min(4096, n - 4096 * b)):
            c, l = 0, 0
            while (l, c) not in table:
                c, l, p = (c << 1) | int(bits[p]), l + 1, p + 1
            out.append(table[(l, c)])
    return np.array(out, np.uint8)


def _canonical_decode_sub(lengths, block_off, sub_bits, payload, n):
    # decoder written from the sub-block index's definition: each 256-byte
    # sub-block is decoded on its own, from the sum of the stated lengths of
    # the sub-blocks before it in its block, and must take exactly its length
    items = sorted((int(l), s) for s, l in enumerate(lengths) if l)
    table, code, prev = {}, 0, items[0][0] if items else 0
    for i, (l, s) in enumerate(items):
        if i:
            code = (code + 1) << (l - prev)
        prev = l
        table[(l, code)] = s
    out = np.zeros(n, np.uint8)
    for b in range(len(block_off) - 1):
        bits = "".join(f"{int(w):032b}" for w in payload[int(block_off[b]): int(block_off[b + 1])])
        for k in range(16):
            start = int(sum(int(v) for v in sub_bits[16 * b: 16 * b + k]))
            p = start
            for i in range(4096 * b + 256 * k, min(4096 * b + 256 * (k + 1), n)):
                c, l = 0, 0
                while (l, c) not in table:
                    c, l, p = (c << 1) | int(bits[p]), l + 1, p + 1
                out[i] = table[(l, c)]
            assert p - start == int(sub_bits[16 * b + k])
    return out


def test_huffman_sub_block_index():
    # the index's closed form: a sub-block's bits are the sum of its bytes'
    # code lengths (0 past the end); the payload does not change with it;
    # decoding from every sub-block's start (the oracle's, and a decoder
    # written from the definition) gives the input back, and an index one
    # bit off anywhere is refused
    rng = np.random.default_rng(101)
    for n in (0, 1, 255, 256, 257, 4095, 4096, 4097, 9000):
        for kind in range(3):
            if kind == 0:
                d = rng.integers(0, 256, n).astype(np.uint8)
            elif kind == 1:
                d = np.clip(np.round(rng.normal(100, 3, n)), 0, 255).astype(np.uint8)
            else:
                d = np.full(n, 42, np.uint8)
            st, ln, off, pay, sub = oracle.huff_encode(d, with_sub=True)
            st0, ln0, off0, pay0 = oracle.huff_encode(d)
            assert st == st0 == oracle.OK and np.array_equal(pay, pay0) and np.array_equal(off, off0)
            nb = (n + 4095) // 4096
            assert sub.size == 16 * nb
            pad = np.zeros(16 * nb * 256, np.int64)
            pad[:n] = ln[d].astype(np.int64) + 0
            want = pad.reshape(-1, 256).sum(axis=1)
            assert np.array_equal(sub.astype(np.int64), want)
            for b in range(nb):
                bits = int(sub[16 * b: 16 * b + 16].astype(np.int64).sum())
                assert int(off[b + 1] - off[b]) == (bits + 31) // 32
            st, back = oracle.huff_decode(ln, off, pay, n, sub)
            assert st == oracle.OK and np.array_equal(back, d)
            if 0 < n <= 4097 and kind < 2:
                assert np.array_equal(_canonical_decode_sub(ln, off, sub, pay, n), d)
            if n > 0:
                for j in (0, int(rng.integers(0, (n - 1) // 256 + 1))):
                    for delta in (1, -1):
                        bad = sub.astype(np.int64)
                        bad[j] += delta
                        if bad[j] < 0:
                            continue
                        assert oracle.huff_decode(ln, off, pay, n, bad.astype(np.uint16))[0] == oracle.EINVAL


def test_huffman_hand_examples():
    g = json.load(open(os.path.join(GOLDEN, "hand_huffman.json")))
    for c in g["cases"]:
        st, ln, off, pay = oracle.huff_encode(np.array(c["data"], np.uint8))
        assert st == oracle.OK
        assert {str(i): int(ln[i]) for i in range(256) if ln[i]} == c["lengths"], c
        assert off.tolist() == c["block_off"] and pay.tolist() == c["payload"], c


def test_huffman_lengths_optimal_and_complete():
    rng = np.random.default_rng(98)
    for trial in range(200):
        k = int(rng.integers(2, 257))
        counts = np.zeros(256, np.uint64)
        syms = rng.choice(256, k, replace=False)
        kind = trial % 3
        if kind == 0:
            counts[syms] = rng.integers(1, 1000, k)
        elif kind == 1:
            counts[syms] = (rng.pareto(1.2, k) * 100).astype(np.uint64) + 1
        else:
            counts[syms] = rng.integers(1, 4, k)  # many ties
        st, ln = oracle.huff_lengths(counts)
        assert st == oracle.OK
        used = counts > 0
        assert np.all((ln > 0) == used)
        kraft = sum(2.0 ** -int(l) for l in ln[used])
        assert kraft == 1.0  # a complete prefix code
        assert int((counts.astype(object) * ln.astype(object)).sum()) == _huffman_cost(counts)


def test_huffman_closed_forms():
    st, ln = oracle.huff_lengths(np.full(256, 5, np.uint64))
    assert np.all(ln == 8)                       # uniform over 256 bytes: 8 bits
    c = np.zeros(256, np.uint64)
    c[[10, 20, 30, 40, 50]] = [16, 8, 4, 2, 2]   # dyadic: lengths -log2(p)
    st, ln = oracle.huff_lengths(c)
    assert [int(ln[i]) for i in (10, 20, 30, 40, 50)] == [1, 2, 3, 4, 4]
    c = np.zeros(256, np.uint64)
    c[200] = 9
    assert oracle.huff_lengths(c)[1][200] == 1    # one used byte: one bit
    # Fibonacci counts force a depth beyond 32 bits: refused
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    c = np.zeros(256, np.uint64)
    c[:40] = fib
    assert oracle.huff_lengths(c)[0] == oracle.ERANGE


def test_huffman_round_trip_and_format():
    rng = np.random.default_rng(99)
    for n in (0, 1, 5, 4095, 4096, 4097, 20000):
        for kind in range(3):
            if kind == 0:
                d = rng.integers(0, 256, n).astype(np.uint8)
            elif kind == 1:
                d = np.clip(np.round(rng.normal(100, 3, n)), 0, 255).astype(np.uint8)
            else:
                d = np.full(n, 42, np.uint8)
            st, ln, off, pay = oracle.huff_encode(d)
            assert st == oracle.OK and len(off) == (n + 4095) // 4096 + 1
            st, back = oracle.huff_decode(ln, off, pay, n)
            assert st == oracle.OK and np.array_equal(back, d)
            if 0 < n <= 4097:
                assert np.array_equal(_canonical_decode(ln, off, pay, n), d)
            h = np.bincount(d, minlength=256)
            bits = int((h.astype(np.int64) * ln.astype(np.int64)).sum())
            assert int(off[-1]) * 32 - bits < 32 * max(len(off) - 1, 1)  # padding below a word per block
    # a payload too small: the full size is still reported
    d = rng.integers(0, 256, 10000).astype(np.uint8)
    st, ln, off, pay = oracle.huff_encode(d, cap_words=10)
    assert st == oracle.ETRUNC and int(off[-1]) > 10
    # decoder rejects tables that are no prefix code and offsets past the payload
    st, ln, off, pay = oracle.huff_encode(d)
    bad = ln.copy()
    bad[bad > 0] = 1
    assert oracle.huff_decode(bad, off, pay, d.size)[0] == oracle.EINVAL
    off2 = off.copy()
    off2[-1] += 5
    assert oracle.huff_decode(ln, off2, pay, d.size)[0] == oracle.EINVAL


def test_per_slice_threshold():
    # per-slice Otsu (each z-slice thresholded on its own, as the paper does
    # per 2-D image): identical slices give the global split on every slice
    rng = np.random.default_rng(100)
    img = np.where(rng.random((24, 40)) < 0.3, 0.8, 0.2) + rng.normal(0, 0.02, (24, 40))
    vol = np.repeat(img[None], 5, axis=0).astype(np.float32)
    g = oracle.fused(vol, "abs", 1e-3, "otsu", 0.0, 6, "min_size", 1)
    s = oracle.fused(vol, "abs", 1e-3, "otsu_slice", 0.0, 6, "min_size", 1)
    assert s["status"] == 0 and s["info"].flags & oracle.FLAG_SLICE
    assert np.all(s["slice_thr"] == g["info"].otsu_bin)
    assert s["info"].n_mask == g["info"].n_mask
    # a brightness drift across z: one global split misses the dim slices,
    # per-slice splits find the object in every slice
    nz = 6
    obj = np.zeros((nz, 24, 40), bool)
    obj[:, 6:18, 10:30] = True
    drift = np.linspace(0.0, 0.6, nz)[:, None, None]
    vol = (np.where(obj, 0.35, 0.05) + drift + rng.normal(0, 0.01, obj.shape)).astype(np.float32)
    s = oracle.fused(vol, "abs", 1e-3, "otsu_slice", 0.0, 6, "min_size", 1)
    g = oracle.fused(vol, "abs", 1e-3, "otsu", 0.0, 6, "min_size", 1)
    assert s["info"].n_mask == obj.sum() and g["info"].n_mask != obj.sum()
    # each split is Otsu's on that slice's bins (bins from the oracle's codes)
    p = s["params"]
    _, codes, _, _ = oracle.quantize(vol, p)
    bins = ((codes.astype(np.int64) - p.qmin) * 256) // p.K
    for z in range(nz):
        h = np.bincount(bins[z].ravel(), minlength=256).astype(np.uint64)
        assert oracle.otsu(h)[0] == s["slice_thr"][z]
    # a constant slice has no split: empty there, flagged
    vol[2] = 0.5
    s = oracle.fused(vol, "abs", 1e-3, "otsu_slice", 0.0, 6, "min_size", 1)
    assert s["slice_thr"][2] == 255 and s["info"].flags & oracle.FLAG_DEGENERATE


def _span_voxels(vol, rt):
    """Values of every span voxel in stream order (numpy, independent of the oracle's loops)."""
    parts = [vol[r["z"], r["y"], r["xs"]:r["xe"]] for r in rt]
    return np.concatenate(parts) if parts else np.zeros(0, vol.dtype)


def test_section_closed_form_on_grid_points():
    # eb = 2^-10: x = k w gives q = k exactly, so each level is
    # floor(256 (k - qmin) / K) in integers; one FIXED split keeping all
    # voxels of a solid block makes every row one span
    nz, ny, nx = 3, 4, 50
    k = np.arange(nz * ny * nx, dtype=np.int64).reshape(nz, ny, nx) % 997 + 100
    vol = (k.astype(np.float64) / 512.0).astype(np.float32)
    r = oracle.fused(vol, "abs", 2.0 ** -10, "fixed", 0.0, 6, "largest", 1)
    p, info = r["params"], r["info"]
    assert info.n_codes == vol.size and p.qmin == int(k.min()) and p.K == int(k.max() - k.min() + 1)
    st, sec = oracle.section(vol, p, r["rows"], info.n_codes)
    assert st == 0
    want = np.array([(256 * (int(q) - p.qmin)) // p.K for q in k.reshape(-1)], np.uint8)
    assert np.array_equal(sec, want)
    assert sec.min() == 0 and sec.max() == 255


def test_section_agrees_with_the_stream_and_the_threshold():
    # every non-escaped code u of the stream gives the level 256 u // K; the
    # level of a voxel of the kept object is above the Otsu split and that of
    # a voxel outside the mask is not (mask <=> bin > t*)
    w = synth.ellipsoids128()
    c = w.criterion
    r = oracle.fused(w.volume, "abs", 2e-5, c.thr, 0.0, c.connectivity, c.keep, c.min_size)
    p, info, rt = r["params"], r["info"], r["rows"]
    assert info.n_outliers > 0 and p.width_bits == 16
    st, sec = oracle.section(w.volume, p, rt, info.n_codes)
    assert st == 0 and len(sec) == info.n_codes
    u = np.frombuffer(r["stream"].tobytes(), np.uint16).astype(np.int64)
    plain = u != p.esc
    assert np.array_equal(sec[plain].astype(np.int64), (256 * u[plain]) // p.K)
    # the escaped voxels: their own codes, from the values
    x = _span_voxels(w.volume, rt)
    st, q, _, _ = oracle.quantize(x[~plain], p)
    assert np.array_equal(sec[~plain].astype(np.int64), (256 * (q.astype(np.int64) - p.qmin)) // p.K)
    st, qa, _, _ = oracle.quantize(w.volume, p)
    mask = qa >= info.q_thr
    st, labels, keep, _ = oracle.label(mask.astype(np.uint8), c.connectivity, c.keep, c.min_size)
    ks = _span_voxels(keep, rt).astype(bool)
    ms = _span_voxels(mask, rt).astype(bool)
    assert ks.any() and (~ms).any()
    assert np.all(sec[ks] > info.otsu_bin) and np.all(sec[~ms] <= info.otsu_bin)


def test_section_covering_every_voxel_has_the_histogram():
    # spans over whole rows: the levels' counts are the 256-bin histogram
    vol = synth.normal((6, 9, 40), 4242, 0.5, 0.1)
    r = oracle.fused(vol, "abs", 1e-3, "fixed", -1.0, 26, "largest", 1)
    p, info = r["params"], r["info"]
    assert info.n_codes == vol.size
    st, sec = oracle.section(vol, p, r["rows"], info.n_codes)
    assert np.array_equal(np.bincount(sec, minlength=256).astype(np.uint64), r["hist"])


def test_section_refuses_rows_outside_the_volume():
    vol = synth.normal((2, 3, 8), 7, 0.5, 0.1)
    r = oracle.fused(vol, "abs", 1e-3, "fixed", -1.0, 6, "largest", 1)
    rt = r["rows"].copy()
    rt[0]["xe"] = 9
    st, _ = oracle.section(vol, r["params"], rt, r["info"].n_codes)
    assert st == oracle.EINVAL
