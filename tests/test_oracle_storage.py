"""Pins of the oracle's storage emulation and error scales (CPU).

The oracle can evaluate its FP64 sums from attributes and node moments
rounded as a reduced-precision store holds them.  These tests tie that
rounding to definitions other than the oracle's own: the bfloat16 conversion
of a library (PyTorch, round to nearest even) and a brute-force choice among
neighbouring representable values; and they check the consequences the
method fixes: FP32 storage changes results only at FP32 rounding level, BF16
storage stays inside the 2^-8 bound that Cauchy-Schwarz gives for a relative
perturbation of every dipole, and keeping every level in FP32 with
BF16-exact attributes reproduces FP32 storage bit for bit.
"""
import numpy as np
import pytest

import workloads
from parity import norm_err_all


def _bf16_neighbours_nearest(v):
    """Nearest bfloat16 to the FP32 value v by brute force: the two
    bfloat16 values that bracket v (v's bits with the low 16 cleared, and the
    next one away from zero), ties to the even significand."""
    u = np.array([v], np.float32).view(np.uint32)[0]
    lo = np.uint32(u & 0xFFFF0000)
    hi = np.uint32(lo + 0x10000)
    a = float(np.array([lo], np.uint32).view(np.float32)[0])
    b = float(np.array([hi], np.uint32).view(np.float32)[0])
    da, db = abs(float(v) - a), abs(float(v) - b)
    if da < db:
        return a
    if db < da:
        return b
    return a if ((lo >> 16) & 1) == 0 else b


def test_round_bf16_matches_library_conversion(orc):
    import torch
    rng = np.random.default_rng(0)
    v = (rng.standard_normal(20000) * 10.0 ** rng.integers(-38, 38, 20000)).astype(np.float32)
    edge = np.array([1.0, 1.00390625, 1.005859375, 1.001953125, -1.001953125, 3.0e38, 1e-40, -2.3e-39,
                     0.0, 1.0078125, 1.01171875, 2.0 ** -126, 2.0 ** -133 * 1.5], np.float32)
    v = np.concatenate([v[np.isfinite(v)], edge])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([orc.round_bf16(a) for a in v])
    assert np.array_equal(got, ref)


def test_round_bf16_is_the_nearest_value(orc):
    rng = np.random.default_rng(1)
    # values at and around ties: low 16 bits 0x8000 exactly, and one off
    base = rng.integers(0x3F800000, 0x40000000, 300).astype(np.uint32) & np.uint32(0xFFFF0000)
    bits = np.concatenate([base | 0x8000, base | 0x7FFF, base | 0x8001, base,
                           rng.integers(0x00800000, 0x7F000000, 3000).astype(np.uint32)])
    v = bits.view(np.float32)
    for a in np.concatenate([v, -v]):
        assert orc.round_bf16(a) == _bf16_neighbours_nearest(a), a


@pytest.fixture(scope="module")
def small(orc):
    p, n, A, mu = workloads.sfm_cloud(6000, 300, 3)
    T = orc.Tree(p, n, A, mu, 8)
    x = workloads.sphere_queries(1500, 4)
    return p, n, A, mu, T, x


def test_stored_values_are_the_rounded_ones(orc, small):
    p, n, A, mu, T, x = small
    ex = T.export()
    for L in (-1, 1, 3, 100):
        T.set_storage("bf16", L)
        Ds, mus = T.export_stored()
        lev = ex["nodes"][:, 0]
        f32 = Ds.astype(np.float32)
        assert np.array_equal(f32.astype(np.float64), Ds)  # representable in FP32
        low = f32.view(np.uint32) & 0xFFFF
        deep = lev > L
        assert np.all(low[deep] == 0)  # bfloat16 values below the FP32 levels
        # the FP32 rounding of the FP64 moment, then the nearest bfloat16
        r32 = ex["D"].astype(np.float32)
        assert np.array_equal(f32[~deep], r32[~deep])
        sample = np.flatnonzero(deep.repeat(Ds.shape[1] * 3))[::97]
        for k in sample:
            assert Ds.reshape(-1)[k] == _bf16_neighbours_nearest(r32.reshape(-1)[k])
        # attributes: bfloat16 of the FP32 inputs, sorted order
        perm = ex["perm"]
        assert np.array_equal(mus, np.array([[orc.round_bf16(a) for a in row] for row in mu[perm]]))
    T.set_storage("exact")
    Ds, mus = T.export_stored()
    assert np.array_equal(Ds, ex["D"]) and np.array_equal(mus, mu[ex["perm"]].astype(np.float64))


def test_fp32_storage_moves_results_by_fp32_rounding(orc, small):
    p, n, A, mu, T, x = small
    T.set_storage("exact")
    ref = T.query(x, 2.0, 0.02)
    T.set_storage("fp32")
    got = T.query(x, 2.0, 0.02)
    T.set_storage("exact")
    assert norm_err_all(got["f"], ref["f"], ref["sf"]).max() <= 1.2e-7
    assert norm_err_all(got["g"], ref["g"], ref["sg"]).max() <= 1.2e-7


@pytest.mark.parametrize("scale", ["mass", "moment"])
def test_bf16_storage_inside_the_rounding_bound(orc, small, scale):
    """|D' - D| <= 2^-8 |D| componentwise, so |dD . d| <= 2^-8 |D| |d| per term:
    normalised errors stay below 2^-8 under either scale."""
    p, n, A, mu, T, x = small
    T.set_scale(scale)
    T.set_storage("exact")
    ref = T.query(x, 1.0, 0.02)
    adj0 = T.adjoint(x, 1.0, 0.02, workloads.cotangents(x.shape[0], mu.shape[1], 7))
    T.set_storage("bf16", -1)
    got = T.query(x, 1.0, 0.02)
    adj = T.adjoint(x, 1.0, 0.02, workloads.cotangents(x.shape[0], mu.shape[1], 7))
    T.set_storage("exact")
    T.set_scale("mass")
    ef = norm_err_all(got["f"], ref["f"], ref["sf"])
    eg = norm_err_all(got["g"], ref["g"], ref["sg"])
    assert ef.max() <= 2.0 ** -8 * (1 + 1e-6) and eg.max() <= 2.0 ** -8 * (1 + 1e-6)
    assert ef.max() > 1e-5  # the emulation does change results
    # dL/dmu is linear in the cotangents only: unchanged by storage
    assert np.array_equal(adj["dmu"], adj0["dmu"])
    assert norm_err_all(adj["dx"], adj0["dx"], adj0["sdx"]).max() <= 2.0 ** -8 * (1 + 1e-6)


def test_all_levels_fp32_and_bf16_exact_attributes_equal_fp32_storage(orc):
    p, n, A, _ = workloads.sphere_cloud(3000, 8)
    rng = np.random.default_rng(9)
    mu = (rng.integers(-64, 64, size=(3000, 3)) / 16.0).astype(np.float32)  # exact in bfloat16
    T = orc.Tree(p, n, A, mu, 8)
    x = workloads.sphere_queries(800, 10)
    T.set_storage("bf16", 100)
    a = T.query(x, 2.0, 0.05)
    T.set_storage("fp32")
    b = T.query(x, 2.0, 0.05)
    assert np.array_equal(a["f"], b["f"]) and np.array_equal(a["g"], b["g"])


def test_storage_survives_new_attributes(orc, small):
    p, n, A, mu, T, x = small
    T.set_storage("bf16", 2)
    mu2 = np.random.default_rng(11).standard_normal(mu.shape).astype(np.float32)
    T.set_attrs(mu2)
    Ds, mus = T.export_stored()
    ex = T.export()
    deep = ex["nodes"][:, 0] > 2
    assert np.all(Ds.astype(np.float32).view(np.uint32)[deep] & 0xFFFF == 0)
    T.set_attrs(mu)
    T.set_storage("exact")


def test_moment_scale_is_tighter(orc, small):
    """|D_t| <= sum |D_m| (triangle inequality): the moment scale never exceeds
    the mass scale, and equals it where no node is taken as far field."""
    p, n, A, mu, T, x = small
    T.set_storage("exact")
    a = T.query(x, 2.0, 0.02)
    T.set_scale("moment")
    b = T.query(x, 2.0, 0.02)
    big = T.query(x, 1e6, 0.02)  # every node opened: points only
    T.set_scale("mass")
    big0 = T.query(x, 1e6, 0.02)
    assert np.all(b["sf"] <= a["sf"] * (1 + 1e-12)) and np.all(b["sg"] <= a["sg"] * (1 + 1e-12))
    assert np.array_equal(a["f"], b["f"])
    assert np.any(b["sf"] < 0.9 * a["sf"])
    # (single-point nodes, r = 0, can still be far: |D| = A |mu| |n| there)
    assert np.allclose(big["sf"], big0["sf"], rtol=1e-12, atol=0)
