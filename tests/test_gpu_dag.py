"""Layered DAG execution on the GPU against the oracle (ops one at a time).

Every execution mode (one launch per op, one fused launch per level, replay
of a captured hipGraph) and every dispatch policy (static threshold, learned,
all-GPU, all-CPU) must give the oracle's node shares bit for bit and the
oracle's MAC-check sigma.
"""
import numpy as np
import pytest
import torch

import oracle.fast as F
from oracle.pipelines import dag_run
from tests._util import host, ints_of_sigma
from workloads import ARR_DAG_IN0, ARR_DAG_TRIPLE0, P61
from workloads.dag import make_dag, to_op_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def build(dag, seed):
    from paper_2512_11112_amd import spdz as S
    f = F.Field(dag.p)
    al = f.alpha_shares(dag.n_parties, seed)
    ctx = S.Context(dag.n_parties, dag.p, ints_of_sigma(al), seed)
    g = S.Dag(ctx, [dag.in_width, dag.in_width], to_op_table(dag))
    g.deal(seed, ARR_DAG_IN0, ARR_DAG_TRIPLE0)
    return ctx, g


def check_nodes(g, ref, nodes):
    for nd in nodes:
        got = g.node(nd)
        assert np.array_equal(host(got.val), ref[nd].val), f"node {nd} values"
        assert np.array_equal(host(got.mac), ref[nd].mac), f"node {nd} MACs"


SMALL = dict(depth=10, ops_per_level=40, median=300, sigma=1.5, wmax=5000, in_width=6000)


@pytest.mark.parametrize("n", [2, 3])
def test_dag_modes_and_policies(n):
    from paper_2512_11112_amd import spdz as S
    dag = make_dag(11, P61, n_parties=n, **SMALL)
    ref, ok, sigma = dag_run(dag, seed=5, check_seed=5)
    assert ok
    ctx, g = build(dag, 5)
    assert g.opened_count() == dag.n_opened()
    runs = [(S.MODE_PER_OP, S.POLICY_ALL_GPU), (S.MODE_PER_LEVEL, S.POLICY_ALL_GPU),
            (S.MODE_GRAPH, S.POLICY_ALL_GPU), (S.MODE_GRAPH, S.POLICY_ALL_GPU),
            (S.MODE_PER_LEVEL, S.POLICY_STATIC), (S.MODE_PER_LEVEL, S.POLICY_ALL_CPU)]
    for epoch, (mode, policy) in enumerate(runs):
        print(f"case n={n} mode={mode} policy={policy}", flush=True)
        if policy == S.POLICY_STATIC:
            g.set_threshold(400)   # about half the ops below, half above
        g.run(mode, policy)
        st = g.last_stats()
        if policy == S.POLICY_STATIC:
            assert st["cpu_ops"] > 0 and st["gpu_ops"] > 0
        g.fetch_host_outputs()
        ok_d, sig_d = ctx.spdz_mac_check()
        ref_e, ok_e, sig_e = (ref, ok, sigma) if epoch == 0 else dag_run(dag, seed=5, check_seed=5, epoch=epoch,
                                                                      keep=set())
        assert ok_d and sig_d == ints_of_sigma(sig_e), (mode, policy)
        check_nodes(g, ref, range(dag.n_ops + 2))


def test_dag_learned_policy_and_autotune():
    from paper_2512_11112_amd import spdz as S
    dag = make_dag(12, P61, n_parties=2, **SMALL)
    ref, ok, sigma = dag_run(dag, seed=6, check_seed=6)
    ctx, g = build(dag, 6)
    tile, bpc, ms = g.autotune(max_levels=5)
    assert tile in (512, 1024, 2048, 4096, 8192) and bpc in (2, 4, 8, 16) and ms > 0
    # a cost model that sends small ops to the CPU: random weights, then the output bias decides
    rng = np.random.default_rng(0)
    W = (rng.standard_normal(S.MLP_NPARAM) * 0.05).astype(np.float32)
    W[-2], W[-1] = 8.0, 9.0     # log2 ns: CPU 256 ns, GPU 512 ns per op -> CPU unless transfers cost more
    g.set_cost_model(W, ns_per_byte=0.0, ns_per_copy=0.0)
    g.run(S.MODE_PER_LEVEL, S.POLICY_LEARNED)
    st = g.last_stats()
    assert st["cpu_ops"] > 0
    g.fetch_host_outputs()
    ok_d, sig_d = ctx.spdz_mac_check()
    assert ok_d and sig_d == ints_of_sigma(sigma)
    check_nodes(g, ref, range(dag.n_ops + 2))
    W[-2], W[-1] = 30.0, 1.0    # GPU always
    g.set_cost_model(W, 0.01, 1000.0)
    g.run(S.MODE_GRAPH, S.POLICY_LEARNED)
    assert g.last_stats()["cpu_ops"] == 0
    ok_d, sig_d = ctx.spdz_mac_check()
    _, _, sig1 = dag_run(dag, seed=6, check_seed=6, epoch=1, keep=set())
    assert ok_d and sig_d == ints_of_sigma(sig1)
    check_nodes(g, ref, range(dag.n_ops + 2))


def test_dag_time_level():
    from paper_2512_11112_amd import spdz as S
    ctx = S.Context(2, P61, [1, 2], 0)
    for kind in (0, 1, 2):
        gns, cns, q = S.dag_time_level(ctx, kind, 1 << 10, 64, reps=2)
        assert gns > 0 and cns > 0 and q == 64
    gns, cns, q = S.dag_time_level(ctx, 0, 1 << 22, 500, reps=1)
    assert q == 16


class ArenaCheck:
    """Compares every node the oracle produces with host copies of device node arenas."""

    def __init__(self, dag, arenas):
        widths = np.concatenate(([dag.in_width, dag.in_width], dag.width)).astype(np.int64)
        self.off = np.concatenate(([0], np.cumsum(dag.n_parties * widths)[:-1]))
        self.widths, self.n, self.arenas = widths, dag.n_parties, arenas
        self.bad, self.seen = [], 0

    def __call__(self, node, z):
        o, w = int(self.off[node]), int(self.widths[node])
        for name, (v, m) in self.arenas.items():
            if not (np.array_equal(v[o:o + self.n * w].reshape(self.n, 1, w), z.val) and
                    np.array_equal(m[o:o + self.n * w].reshape(self.n, 1, w), z.mac)):
                self.bad.append((name, node))
        self.seen += 1
        if self.seen % 10000 == 0:
            print(f"oracle: {self.seen} nodes compared", flush=True)


def arena_host(g):
    v, m = g.node_arena()
    out = host(v), host(m)
    del v, m
    torch.cuda.empty_cache()
    return out


@pytest.mark.timeout(1500)
def test_dag_full_size_every_node():
    """The 100k-op, depth-200 workload (seed 0).  Run 1: every op on the GPU, hipGraph replay.
    Run 2: the static policy at MIN_KERNEL_SIZE = 65535 (slice 262140 / 4), where the CPU back
    end runs about 99.4k of the ops.  Every node of both runs (values and MAC shares) equals the
    oracle's, and so do both MAC checks' sigma (check numbers 0 and 1)."""
    from paper_2512_11112_amd import spdz as S
    dag = make_dag(0, P61)
    assert dag.n_ops == 100000
    ctx, g = build(dag, 0)
    print("case full-size DAG: graph mode, all on the GPU", flush=True)
    g.run(S.MODE_GRAPH, S.POLICY_ALL_GPU)
    ok0, sig0 = ctx.spdz_mac_check()
    arenas = {"graph": arena_host(g)}
    print("case full-size DAG: static policy at 65535", flush=True)
    g.set_threshold(65535)
    g.run(S.MODE_PER_LEVEL, S.POLICY_STATIC)
    st = g.last_stats()
    assert st["cpu_ops"] > 99000, st
    g.fetch_host_outputs()
    ok1, sig1 = ctx.spdz_mac_check()
    arenas["static"] = arena_host(g)
    g.close()
    ctx.close()
    print("oracle", flush=True)
    chk = ArenaCheck(dag, arenas)
    _, ok, sigma, more = dag_run(dag, seed=0, check_seed=0, keep=set(), on_node=chk, more_epochs=(1,))
    assert chk.seen == dag.n_ops + 2
    assert not chk.bad, chk.bad[:10]
    assert ok and ok0 and sig0 == ints_of_sigma(sigma)
    assert more[1][0] and ok1 and sig1 == ints_of_sigma(more[1][1])
