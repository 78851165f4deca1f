"""Precision study at 4,194,304 points, FP32- vs BF16-stored attributes and
moments (FP64 accumulation of the top-level moments, since M >= 4,194,304),
beta in {1, 2, 4}, on two clouds: sphere-4m (points on the unit sphere, 32,768
queries U([-1.5,1.5]^3), eps = 0.05) and sfm-4m (the 1M scene's SfM-like
distributions at 4M points, 32,768 samples on 256 rays of its camera,
eps = 0.01414).  Errors are normalised by the per-query absolute sums and
reported against the FP64 oracle's Barnes-Hut result (same decisions) and
against the FP64 direct sum on a query subset (which adds the Barnes-Hut
approximation error of Sec. 6.1)."""
import json
import os

import numpy as np
import pytest

import workloads
from parity import TOL_BF16, TOL_FP32, norm_err_all, to_dev, to_host

pytestmark = pytest.mark.gpu

M = 4_194_304
EPS = 0.05


@pytest.fixture(scope="module")
def sphere4m(orc):
    import torch
    import paper_2405_16788_amd as P
    P.load()
    assert torch.cuda.is_available()
    p, n, A, mu = workloads.sphere_cloud(M, 20)
    x = workloads.sphere_queries(32768, 21)
    print(f"[precision] oracle tree M={M}", flush=True)
    T = orc.Tree(p, n, A, mu, 16)
    sub = x[np.random.default_rng(22).choice(x.shape[0], 384, replace=False)]
    print("[precision] oracle direct sum on 384 queries", flush=True)
    direct = orc.direct(p, n, A, mu, sub, EPS)
    return P, T, (p, n, A, mu, x, sub), direct


def test_sphere_4m_precision_table(sphere4m):
    P, T, (p, n, A, mu, x, sub), direct = sphere4m
    dev = to_dev(p, n, A, mu, x, sub)
    table = []
    for storage in ("fp32", "bf16"):
        tree = P.dps_build(*dev[:4], leaf_size=16, storage=storage)
        info = P.dps_tree_info(tree)
        for beta in (1.0, 2.0, 4.0):
            ref = T.query(x, beta, EPS)
            f, g = P.dps_query(tree, dev[4], beta, EPS)
            counts = P.dps_query_counts(tree, dev[4], beta)
            assert np.array_equal(to_host(counts), ref["counts"])
            ef = norm_err_all(to_host(f), ref["f"], ref["sf"])
            eg = norm_err_all(to_host(g), ref["g"], ref["sg"])
            fs, gs = P.dps_query(tree, dev[5], beta, EPS)
            bh_sub = T.query(sub, beta, EPS)
            df_ = norm_err_all(to_host(fs), direct["f"], direct["sf"])
            dg_ = norm_err_all(to_host(gs), direct["g"], direct["sg"])
            bf_ = norm_err_all(bh_sub["f"], direct["f"], direct["sf"])
            row = {"storage": storage, "beta": beta, "nodes": info["n_nodes"],
                   "vs_bh_f_max": float(ef.max()), "vs_bh_f_p999": float(np.percentile(ef, 99.9)),
                   "vs_bh_g_max": float(eg.max()),
                   "vs_direct_f_max": float(df_.max()), "vs_direct_f_mean": float(df_.mean()),
                   "vs_direct_g_max": float(dg_.max()),
                   "oracle_bh_vs_direct_f_max": float(bf_.max()),
                   "visits_per_query": float(ref["counts"][:, 0].mean())}
            table.append(row)
            print("[precision] " + json.dumps(row), flush=True)
            tol = TOL_BF16 if storage == "bf16" else TOL_FP32
            # BF16: the hard bound holds for every query; the 2e-3 percentile
            # target needs many far sources per query (beta = 1 visits ~7 nodes
            # here, so single sources dominate) and is reported in the table
            assert row["vs_bh_f_max"] <= tol and row["vs_bh_g_max"] <= tol
            # the GPU result differs from the direct sum by the BH error plus
            # at most the storage error
            assert row["vs_direct_f_max"] <= row["oracle_bh_vs_direct_f_max"] + tol
        P.dps_destroy(tree)
    # larger beta: never less accurate on average against the direct sum
    for st in ("fp32", "bf16"):
        m = [r["vs_direct_f_mean"] for r in table if r["storage"] == st]
        assert m[0] >= m[1] >= m[2]
    out = os.environ.get("DPS_PRECISION_TABLE")
    if out:
        with open(out, "w") as fh:
            json.dump(table, fh, indent=1)


@pytest.fixture(scope="module")
def sfm4m(orc):
    import torch
    import paper_2405_16788_amd as P
    P.load()
    assert torch.cuda.is_available()
    p, n, A, mu = workloads.sfm_cloud(workloads.SFM_4M_SURFACE, workloads.SFM_4M_OUTLIERS, 40)
    assert p.shape[0] == M
    _, x = workloads.pixel_ray_samples(workloads.sfm_camera(11), 512, 512, 128, 41, 256, 42)
    print(f"[precision] sfm-4m oracle tree M={M}", flush=True)
    T = orc.Tree(p, n, A, mu, 16)
    sub = x[np.random.default_rng(43).choice(x.shape[0], 256, replace=False)]
    print("[precision] sfm-4m oracle direct sum on 256 queries", flush=True)
    direct = orc.direct(p, n, A, mu, sub, EPS_SFM)
    return P, T, (p, n, A, mu, x, sub), direct


EPS_SFM = 0.01414


def test_sfm_4m_precision_table(sfm4m):
    P, T, (p, n, A, mu, x, sub), direct = sfm4m
    dev = to_dev(p, n, A, mu, x, sub)
    for storage in ("fp32", "bf16"):
        tree = P.dps_build(*dev[:4], leaf_size=16, storage=storage)
        for beta in (1.0, 2.0, 4.0):
            ref = T.query(x, beta, EPS_SFM)
            f, g = P.dps_query(tree, dev[4], beta, EPS_SFM)
            counts = P.dps_query_counts(tree, dev[4], beta)
            assert np.array_equal(to_host(counts), ref["counts"])
            ef = norm_err_all(to_host(f), ref["f"], ref["sf"])
            eg = norm_err_all(to_host(g), ref["g"], ref["sg"])
            fs, gs = P.dps_query(tree, dev[5], beta, EPS_SFM)
            bh_sub = T.query(sub, beta, EPS_SFM)
            df_ = norm_err_all(to_host(fs), direct["f"], direct["sf"])
            bf_ = norm_err_all(bh_sub["f"], direct["f"], direct["sf"])
            row = {"cloud": "sfm-4m", "storage": storage, "beta": beta,
                   "vs_bh_f_max": float(ef.max()), "vs_bh_f_p999": float(np.percentile(ef, 99.9)),
                   "vs_bh_g_max": float(eg.max()), "vs_bh_g_p999": float(np.percentile(eg, 99.9)),
                   "vs_direct_f_max": float(df_.max()), "vs_direct_f_mean": float(df_.mean()),
                   "oracle_bh_vs_direct_f_max": float(bf_.max()),
                   "visits_per_query": float(ref["counts"][:, 0].mean())}
            print("[precision] " + json.dumps(row), flush=True)
            tol = TOL_BF16 if storage == "bf16" else TOL_FP32
            assert row["vs_bh_f_max"] <= tol and row["vs_bh_g_max"] <= tol
            assert row["vs_direct_f_max"] <= row["oracle_bh_vs_direct_f_max"] + tol
        P.dps_destroy(tree)
