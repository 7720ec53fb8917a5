"""HIP graph replay of persistent runs (option use_graphs): the device part of a run is
captured once per job table and replayed; every replay must equal the eager run, with eager
work and synchronisations between the replays, for the R-NW groups and the device
continuation of H_per, and a changed job order or tuning must give the same values."""
import json
import os
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import native

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                     "oracle_values.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("split", [0, 12])
def test_graph_replays_equal_eager(hperm, split):
    items = W.config_n60(3)
    mats = [A for _, A in items]
    want = [int(GOLDEN[n]) for n, _ in items]
    eager = hperm.Context({"split_order": split, "device_expand": 0})
    graph = hperm.Context({"split_order": split, "device_expand": 0, "use_graphs": 1})
    try:
        Je = eager.expand(mats)
        Jg = graph.expand(mats)
        eager.estimate(Je, 16, 1)
        graph.estimate(Jg, 16, 1)
        ref = eager.run(Je, "estimate", True)[0]
        assert ref == want
        small = W.config_n24(range(2))
        for rep in range(4):
            say("graph replay", split, rep)
            for order in ("estimate", "natural", "random"):
                got = graph.run(Jg, order, True)[0]
                assert got == ref, (rep, order)
            # eager work on the graph's context and elsewhere, with synchronisations, between replays
            assert graph.permanent_batch(small) == [int(GOLDEN[f"cubic24_seed{s}"]) for s in range(2)]
            assert eager.run(Je, "natural", True)[0] == ref
            torch.cuda.synchronize()
        # per-job results are never captured: an eager run on the same table
        _, pj, _ = graph.run(Jg, "natural", True, per_job=True)
        assert sum(pj) == sum(ref) and pj == eager.run(Je, "natural", True, per_job=True)[1]
        assert graph.run(Jg, "estimate", True)[0] == ref
    finally:
        eager.close()
        graph.close()


def test_graph_after_tuning_and_new_tables(hperm):
    rng = np.random.default_rng(9)
    mats = [W.permutation_union_matrix(int(m), 4, 500 + i, 1, 5) for i, m in enumerate(rng.integers(16, 25, size=30))]
    want = native.hper_batch(mats, threads=8)
    c = hperm.Context({"split_order": 0, "device_expand": 0, "use_graphs": 1})
    try:
        J = c.jobs_from_dense(mats)
        first = [c.run(J, "natural", True)[0] for _ in range(3)]
        c.autotune(J)
        tuned = [c.run(J, "natural", True)[0] for _ in range(3)]
        J2 = c.jobs_from_dense(mats[::-1])
        other = [c.run(J2, "natural", True)[0] for _ in range(2)]
        again = c.run(J, "natural", True)[0]
    finally:
        c.close()
    for got in first + tuned + [again]:
        assert got == want
    for got in other:
        assert got == want[::-1]
