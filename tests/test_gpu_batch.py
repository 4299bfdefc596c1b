"""Batching of uneven problems (one multi-problem launch per time block,
captured in a hipGraph, autotuned): every problem of a batch equals its
own single-problem run bit for bit and matches the oracle."""

import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_helpers import inputs_as, problem_pair, rel_energy_err, to_np

pytestmark = pytest.mark.gpu


def _batch_workloads():
    # uneven fine grids 64^2, 96^2, 80^2; slices, steps and media differ
    return [W.grf2d(n=64, N=8, K=2, T=0.25, seed=0),
            W.grf2d(n=96, N=8, K=2, T=0.25, seed=1),
            W.grf2d(n=80, N=6, K=2, T=0.2, seed=2)]


def _solver(ws, K, tol=1e-6):
    import paper_1905_00473_amd as pw
    probs = [problem_pair(w, max_iters=K, tol=tol)[0] for w in ws]
    s = pw.Solver(probs)
    for i, w in enumerate(ws):
        u0, p0 = inputs_as(w, w.dtype)
        s.set_medium(w.c, prob=i)
        s.set_initial(u0, p0, prob=i)
    return s


def test_batch_equals_single_runs_bitwise(tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("PW_TUNE_CACHE", str(tmp_path / "tune.txt"))
    ws = _batch_workloads()
    K = 2
    sb = _solver(ws, K)
    sb.run_batch(K)
    info = sb.batch_info()
    assert info["depth"] in (4, 8) and info["rows_per_stream"] in (64, 128, 256)
    for i, w in enumerate(ws):
        s1 = _solver([w], K)
        s1.run(K)
        for n in range(w.N + 1):
            ub, pb = sb.state(n, prob=i)
            u1, p1 = s1.state(n)
            assert torch.equal(ub, u1) and torch.equal(pb, p1), (i, n)
        assert sb.residuals(prob=i) == s1.residuals()
    # replaying the captured graph gives the same answer again
    first = [sb.state(ws[i].N, prob=i)[0].clone() for i in range(len(ws))]
    sb.run_batch(K)
    for i in range(len(ws)):
        assert torch.equal(first[i], sb.state(ws[i].N, prob=i)[0])


def test_batch_matches_oracle(tmp_path, monkeypatch):
    monkeypatch.setenv("PW_TUNE_CACHE", str(tmp_path / "tune.txt"))
    ws = _batch_workloads()
    K = 2
    sb = _solver(ws, K)
    sb.run_batch(K)
    for i, w in enumerate(ws):
        _, Q = problem_pair(w, max_iters=K, tol=1e-6)
        u0, p0 = inputs_as(w, w.dtype)
        ref = O.theta_parareal(Q, w.c, u0, p0, K)
        for n in range(1, w.N + 1):
            u, p = sb.state(n, prob=i)
            e = rel_energy_err(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                               Q.dx_fine)
            assert e < 1e-5, (i, n, e)


def test_autotuner_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("PW_TUNE_CACHE", str(path))
    ws = _batch_workloads()
    s = _solver(ws, 1)
    s.run_batch(1)
    a = s.batch_info()
    assert not a["from_cache"] and a["tune_ms"] > 0
    text = path.read_text()
    assert "64x64N8" in text and "96x96N8" in text
    s2 = _solver(ws, 1)
    s2.run_batch(1)
    b = s2.batch_info()
    assert b["from_cache"]
    assert (a["depth"], a["rows_per_stream"]) == (b["depth"],
                                                  b["rows_per_stream"])
    assert s2.batch_fine_sweeps(2) > 0


def test_batch_rejects_mixed_problems():
    import paper_1905_00473_amd as pw
    w2 = W.grf2d(n=64, N=8, K=1, T=0.25, seed=0)
    w1 = W.wave1d()
    s = _solver([w2, w1], 1)
    with pytest.raises(pw.PwError):
        s.run_batch(1)


def test_batch_with_sampling_equals_single_runs(tmp_path, monkeypatch):
    """Random subsampling set on some problems of a batch: each problem
    still equals its own single-problem run with the same table bit for
    bit; a variant other than Algorithm 3 is refused by batched runs."""
    import paper_1905_00473_amd as pw
    import torch
    monkeypatch.setenv("PW_TUNE_CACHE", str(tmp_path / "tune.txt"))
    ws = _batch_workloads()
    K = 2
    tables = [W.sample_columns(ws[0].N, 3, K, seed=4), None,
              W.sample_columns(ws[2].N, 5, K, seed=6)]
    sb = _solver(ws, K)
    for i, t in enumerate(tables):
        sb.set_sampling(t, prob=i)
    sb.run_batch(K)
    for i, w in enumerate(ws):
        s1 = _solver([w], K)
        s1.set_sampling(tables[i])
        s1.run(K)
        for n in range(w.N + 1):
            ub, pb = sb.state(n, prob=i)
            u1, p1 = s1.state(n)
            assert torch.equal(ub, u1) and torch.equal(pb, p1), (i, n)
        assert sb.residuals(prob=i) == s1.residuals()
        s1.close()
    sb.set_variant("plain", prob=1)
    with pytest.raises(pw.PwError, match="Algorithm 3 only"):
        sb.run_batch(K)
    sb.close()
