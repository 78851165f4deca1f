"""Precision study at 4,194,304 points, FP32- vs BF16-stored attributes and
moments, beta in {1, 2, 4}, on two clouds: sphere-4m (points on the unit
sphere, 32,768 queries U([-1.5,1.5]^3), eps = 0.05) and sfm-4m (the 1M
scene's SfM-like distributions at 4M points, 32,768 samples on 256 rays of its
camera, eps = 0.01414).

The refit accumulates the top-level moments (depth <= 3) in FP64 at this size
and compensated FP32 below; BF16 storage keeps the depth <= 3 moments in FP32
(a query far from the geometry takes a few large nodes as its whole far field,
so their rounding would not average out) and everything else in bfloat16.

Errors are normalised by each result's absolute scale and reported against
the FP64 oracle's Barnes-Hut result (same decisions) under two scales of a
node term -- its absolute mass (the default) and the magnitude of its own
moment |D_t| (stricter where moments cancel) -- with the normwise error
||gpu - oracle||_2 / ||oracle||_2 beside them; BF16 also against the oracle
evaluated from identically rounded values (FP32 bar), and both against the
FP64 direct sum on a query subset (which adds the Barnes-Hut approximation
error of Sec. 6.1).
"""
import json
import os

import numpy as np
import pytest

import workloads
from parity import TARGET_BF16, TOL_BF16, TOL_FP32, norm_err_all, normwise, to_dev, to_host

pytestmark = pytest.mark.gpu

M = 4_194_304
EPS = 0.05
EPS_SFM = 0.01414
FP32_LEVELS = 3


def _make(orc, cloud):
    import torch
    import paper_2405_16788_amd as P
    P.load()
    assert torch.cuda.is_available()
    if cloud == "sphere-4m":
        p, n, A, mu = workloads.sphere_cloud(M, 20)
        x = workloads.sphere_queries(32768, 21)
        sub_seed, n_sub = 22, 384
    else:
        p, n, A, mu = workloads.sfm_cloud(workloads.SFM_4M_SURFACE, workloads.SFM_4M_OUTLIERS, 40)
        assert p.shape[0] == M
        _, x = workloads.pixel_ray_samples(workloads.sfm_camera(11), 512, 512, 128, 41, 256, 42)
        sub_seed, n_sub = 43, 256
    print(f"[precision] {cloud}: oracle tree M={M}", flush=True)
    T = orc.Tree(p, n, A, mu, 16)
    sub = x[np.random.default_rng(sub_seed).choice(x.shape[0], n_sub, replace=False)]
    eps = EPS if cloud == "sphere-4m" else EPS_SFM
    print(f"[precision] {cloud}: oracle direct sum on {n_sub} queries", flush=True)
    direct = orc.direct(p, n, A, mu, sub, eps)
    return P, T, (p, n, A, mu, x, sub), direct, eps


@pytest.fixture(scope="module")
def sphere4m(orc):
    return _make(orc, "sphere-4m")


@pytest.fixture(scope="module")
def sfm4m(orc):
    return _make(orc, "sfm-4m")


def _table(cloud, setup):
    P, T, (p, n, A, mu, x, sub), direct, eps = setup
    dev = to_dev(p, n, A, mu, x, sub)
    table = []
    for storage in ("fp32", "bf16"):
        tree = P.dps_build(*dev[:4], leaf_size=16, storage=storage)
        for beta in (1.0, 2.0, 4.0):
            T.set_storage("exact")
            T.set_scale("mass")
            ref = T.query(x, beta, eps)
            T.set_scale("moment")
            ref_m = T.query(x, beta, eps)
            T.set_scale("mass")
            f, g = P.dps_query(tree, dev[4], beta, eps)
            assert np.array_equal(to_host(P.dps_query_counts(tree, dev[4], beta)), ref["counts"])
            f, g = to_host(f), to_host(g)
            ef = norm_err_all(f, ref["f"], ref["sf"])
            eg = norm_err_all(g, ref["g"], ref["sg"])
            efm = norm_err_all(f, ref["f"], ref_m["sf"])
            egm = norm_err_all(g, ref["g"], ref_m["sg"])
            fs, gs = P.dps_query(tree, dev[5], beta, eps)
            bh_sub = T.query(sub, beta, eps)
            df_ = norm_err_all(to_host(fs), direct["f"], direct["sf"])
            bf_ = norm_err_all(bh_sub["f"], direct["f"], direct["sf"])
            row = {"cloud": cloud, "storage": storage, "beta": beta,
                   "f_max": float(ef.max()), "f_p999": float(np.percentile(ef, 99.9)),
                   "g_max": float(eg.max()), "g_p999": float(np.percentile(eg, 99.9)),
                   "f_max_moment_scale": float(efm.max()), "g_max_moment_scale": float(egm.max()),
                   "f_normwise": normwise(f, ref["f"]), "g_normwise": normwise(g, ref["g"]),
                   "vs_direct_f_max": float(df_.max()), "vs_direct_f_mean": float(df_.mean()),
                   "oracle_bh_vs_direct_f_max": float(bf_.max()),
                   "visits_per_query": float(ref["counts"][:, 0].mean())}
            if storage == "bf16":
                T.set_storage("bf16", FP32_LEVELS)
                emu = T.query(x, beta, eps)
                T.set_storage("exact")
                ee = np.concatenate([norm_err_all(f, emu["f"], emu["sf"]), norm_err_all(g, emu["g"], emu["sg"])])
                row["vs_emulated_max"] = float(ee.max())
                row["vs_emulated_over_1e-5"] = int((ee > TOL_FP32).sum())
            table.append(row)
            print("[precision] " + json.dumps(row), flush=True)
            if storage == "fp32":
                assert max(row["f_max"], row["g_max"]) <= TOL_FP32
                assert max(row["f_max_moment_scale"], row["g_max_moment_scale"]) <= TOL_FP32
            else:
                # the stated BF16 bar, for every query, under either scale
                assert max(row["f_max"], row["g_max"]) <= TARGET_BF16
                assert max(row["f_max_moment_scale"], row["g_max_moment_scale"]) <= TARGET_BF16
                # the arithmetic of the stored values: FP32 bar against the
                # oracle fed the same rounded values (rounding-boundary flips
                # of the stored moments, if any, touch very few results)
                assert row["vs_emulated_over_1e-5"] <= ee.size // 1000 and row["vs_emulated_max"] <= TOL_BF16
            # against the direct sum: the BH error plus at most the storage error
            assert row["vs_direct_f_max"] <= row["oracle_bh_vs_direct_f_max"] + (
                TARGET_BF16 if storage == "bf16" else TOL_FP32)
        P.dps_destroy(tree)
    # larger beta: never less accurate on average against the direct sum
    for st in ("fp32", "bf16"):
        m = [r["vs_direct_f_mean"] for r in table if r["storage"] == st]
        assert m[0] >= m[1] >= m[2]
    out = os.environ.get("DPS_PRECISION_TABLE")
    if out:
        with open(f"{out}.{cloud}.json", "w") as fh:
            json.dump(table, fh, indent=1)
    return table


def test_sphere_4m_precision_table(sphere4m):
    _table("sphere-4m", sphere4m)


def test_sfm_4m_precision_table(sfm4m):
    _table("sfm-4m", sfm4m)

