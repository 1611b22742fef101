"""GPU parity of the batched path (tho_batched_*): every problem of a batch
against the CPU oracle of Algorithm 1 (second choice of P), element-wise at
1e-10, on mixed batches with ragged sizes; the full batched workload (4096
problems) is checked on a sample (64 random problems plus the extremes)
against the oracle and against single-problem GPU calls."""

import numpy as np
import pytest
import torch

import tho_workloads as W
from oracle import two_stage as oracle_two_stage, orth_loss, rel_residual

from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def _mixed(seed, count):
    g = np.random.default_rng(seed)
    pairs = []
    for i in range(count):
        k0 = int(g.choice([0, 3, 8, 16, 32, 40, 64]))
        k = int(g.choice([1, 4, 8, 16, 17, 33, 64]))
        n = int(g.integers(k0 + k, 6000))
        V = W.orthonormal(g, n, k0)
        A = g.standard_normal((n, k))
        pairs.append((V, A))
    return pairs


def _check(V, A, Q, R, S, tol=1e-10):
    Qo, Ro, So = oracle_two_stage(V, A)
    assert np.abs(Q - Qo).max() < tol
    assert np.abs(R - Ro).max() < tol * max(1.0, np.abs(Ro).max())
    if So.size:
        assert np.abs(S - So).max() < tol * max(1.0, np.abs(So).max())
    assert orth_loss(V, Q) < 1e-12
    assert rel_residual(V, A, Q, R, S) < 1e-12


@pytest.mark.parametrize("seed,count", [(1, 40), (2, 7), (3, 1)])
def test_batched_mixed(seed, count):
    require_gpu()
    import paper_2602_14449_amd as tho
    pairs = _mixed(seed, count)
    dev = [(to_dev(V), to_dev(A)) for V, A in pairs]
    plan = tho.BatchedPlan(dev)
    out = plan.run()
    print(plan.info())
    for (V, A), (Q, R, S) in zip(pairs, out):
        _check(V, A, to_host(Q), to_host(R), to_host(S))
    # replaying the graph gives the same bits
    first = [to_host(q) for q, _, _ in out]
    out2 = plan.run()
    for a, (q, _, _) in zip(first, out2):
        assert np.array_equal(a, to_host(q))
    plan.close()


def test_batched_edge_shapes():
    require_gpu()
    import paper_2602_14449_amd as tho
    g = np.random.default_rng(5)
    shapes = [(3, 2, 1), (80, 64, 16), (65, 1, 64), (129, 64, 64), (4096, 64, 16), (257, 0, 16), (9000, 16, 0)]
    pairs = [(W.orthonormal(g, n, k0), g.standard_normal((n, k))) for n, k0, k in shapes]
    out = tho.two_stage_batched([(to_dev(V), to_dev(A)) for V, A in pairs])
    for (V, A), (Q, R, S) in zip(pairs, out):
        if A.shape[1] == 0:
            continue
        _check(V, A, to_host(Q), to_host(R), to_host(S))


def test_batched_full_workload_sampled():
    # 4096 problems, n ~ U[2048, 65536], k0 in {8,16,32,64}, k in {4,8,16}
    require_gpu()
    import paper_2602_14449_amd as tho
    pairs = W.batched_gpu(4096)
    plan = tho.BatchedPlan(pairs)
    out = plan.run()
    torch.cuda.synchronize()
    print(plan.info())
    ns = np.array([V.shape[0] for V, _ in pairs])
    g = np.random.default_rng(11)
    sample = set(g.choice(len(pairs), 64, replace=False).tolist())
    sample |= {int(ns.argmax()), int(ns.argmin())}
    for j in sorted(sample):
        V, A = pairs[j]
        Q, R, S = out[j]
        Vh, Ah = to_host(V), to_host(A)
        _check(Vh, Ah, to_host(Q), to_host(R), to_host(S))
        Q1, R1, S1 = tho.two_stage(V, A)
        assert np.abs(to_host(Q1) - to_host(Q)).max() < 1e-10
    plan.close()


_CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, %r)
import paper_2602_14449_amd as tho
import tho_workloads as W
g = np.random.default_rng(4242)
pairs = []
for n, k0, k in [(3001, 8, 4), (5003, 16, 8), (7007, 32, 16)]:
    pairs.append((torch.from_numpy(W.orthonormal(g, n, k0)).cuda(), torch.from_numpy(g.standard_normal((n, k))).cuda()))
plan = tho.BatchedPlan(pairs)
info = plan.info()
print("TUNE", info["tile_rows"], info["workgroups"], info["tuned_ms"])
"""


def test_tuner_cache_file(tmp_path):
    # THO_TUNE_CACHE: the first process tunes and appends its choice to the
    # file; a second process with the same batch reads it back without tuning
    require_gpu()
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, THO_TUNE_CACHE=str(tmp_path / "tune.txt"))
    outs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", _CHILD % root], env=env, capture_output=True, text=True,
                           timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        line = [x for x in r.stdout.splitlines() if x.startswith("TUNE")][-1].split()
        outs.append((int(line[1]), int(line[2]), float(line[3])))
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("tho-batched-v1 ")
    assert outs[0][2] > 0.0 and outs[1][2] == 0.0           # tuned, then read from the file
    assert outs[0][:2] == outs[1][:2]
