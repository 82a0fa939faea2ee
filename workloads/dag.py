"""Seeded layered DAG of batched secret-shared operations.

The paper's runtime executes a data-flow graph whose vector nodes
(AddBatch, MultBatch, ...) carry their lane width (Sec. III-B, "Vectorization
is first-class"); inputs arrive through Load(base, start, count) nodes that
the runtime treats as views onto existing buffers (Sec. III-B, "Normalizing
parameter loads"; Sec. III-C, "Structured Data Movement").  This module draws
the structure of such a graph: which ops exist, their kinds, widths and the
views they read.  It holds no share arithmetic.

Shape of the graph:
  * level 0 holds two dealt input vectors of width `in_width`;
  * levels 1..depth each hold `ops_per_level` ops, kinds drawn i.i.d.
    (Beaver multiplication, addition, multiplication by a public constant);
  * op width w = clip(round(median * exp(sigma * N(0,1))), 1, wmax);
  * operand 1 is the output of a uniformly chosen node of the previous level,
    so the critical path is exactly `depth` ops long;
  * operand 2 (mul/add only) is a uniformly chosen node of any earlier level;
  * an operand is a cyclic view of length w: element j reads
    src[(off + j) mod width(src)] with off uniform in [0, width(src)).
  * a public-constant multiplier is uniform in [1, p).

Node ids: 0 and 1 are the inputs, op k is node k + 2.  Op ids increase level
by level, so op-id order is a topological order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

OP_MUL, OP_ADD, OP_SMUL = 0, 1, 2
OP_NAMES = {OP_MUL: "mul", OP_ADD: "add", OP_SMUL: "smul"}


@dataclass
class Dag:
    seed: int
    p: int
    n_parties: int
    in_width: int
    depth: int
    kind: np.ndarray     # int32 [n_ops]
    level: np.ndarray    # int32 [n_ops], 1..depth
    width: np.ndarray    # int64 [n_ops]
    src1: np.ndarray     # int64 [n_ops] node id
    off1: np.ndarray     # int64 [n_ops]
    src2: np.ndarray     # int64 [n_ops] node id, -1 for smul
    off2: np.ndarray     # int64 [n_ops]
    const: np.ndarray    # uint64 [n_ops] public multiplier (smul), 0 otherwise

    @property
    def n_ops(self) -> int:
        return int(self.kind.shape[0])

    def node_width(self, node: int) -> int:
        return self.in_width if node < 2 else int(self.width[node - 2])

    def level_ops(self, lev: int) -> np.ndarray:
        return np.nonzero(self.level == lev)[0]

    def mul_ops(self) -> np.ndarray:
        return np.nonzero(self.kind == OP_MUL)[0]

    def total_elements(self) -> int:
        return int(self.width.sum())

    def opened_offsets(self) -> np.ndarray:
        """Start index, in the opened-value log, of each Beaver op's d block.

        Every Beaver op opens d (w values) then e (w values); ops enter the log
        in op-id order.  Non-Beaver ops get -1.
        """
        starts = np.full(self.n_ops, -1, dtype=np.int64)
        muls = self.mul_ops()
        sizes = 2 * self.width[muls]
        starts[muls] = np.concatenate(([0], np.cumsum(sizes)[:-1])) if len(muls) else []
        return starts

    def n_opened(self) -> int:
        return int(2 * self.width[self.kind == OP_MUL].sum())


def make_dag(seed: int, p: int, n_parties: int = 2, depth: int = 200,
             ops_per_level: int = 500, probs=(0.6, 0.3, 0.1), median: float = 400.0,
             sigma: float = 2.0, wmax: int = 1 << 20, in_width: int = 1 << 20) -> Dag:
    rng = np.random.Generator(np.random.PCG64(seed))
    n_ops = depth * ops_per_level
    kind = rng.choice(3, size=n_ops, p=np.asarray(probs, dtype=np.float64)).astype(np.int32)
    level = np.repeat(np.arange(1, depth + 1, dtype=np.int32), ops_per_level)
    raw = np.rint(median * np.exp(sigma * rng.standard_normal(n_ops)))
    width = np.clip(raw, 1, wmax).astype(np.int64)

    # node ids of each level: level 0 = {0, 1}; level l = 2 + (l-1)*opl + [0, opl)
    def level_first(lev):
        return 0 if lev == 0 else 2 + (lev - 1) * ops_per_level

    def level_count(lev):
        return 2 if lev == 0 else ops_per_level

    src1 = np.empty(n_ops, dtype=np.int64)
    src2 = np.full(n_ops, -1, dtype=np.int64)
    for lev in range(1, depth + 1):
        sl = slice((lev - 1) * ops_per_level, lev * ops_per_level)
        src1[sl] = level_first(lev - 1) + rng.integers(0, level_count(lev - 1), ops_per_level)
        n_before = 2 + (lev - 1) * ops_per_level  # nodes in levels 0..lev-1
        src2[sl] = rng.integers(0, n_before, ops_per_level)
    src2[kind == OP_SMUL] = -1

    def widths_of(nodes):
        out = np.full(nodes.shape, in_width, dtype=np.int64)
        m = nodes >= 2
        out[m] = width[nodes[m] - 2]
        return out

    off1 = (rng.random(n_ops) * widths_of(src1)).astype(np.int64)
    has2 = src2 >= 0
    off2 = np.zeros(n_ops, dtype=np.int64)
    off2[has2] = (rng.random(int(has2.sum())) * widths_of(src2[has2])).astype(np.int64)
    const = np.zeros(n_ops, dtype=np.uint64)
    n_smul = int((kind == OP_SMUL).sum())
    if p < (1 << 63):
        const[kind == OP_SMUL] = rng.integers(1, p, n_smul, dtype=np.uint64)
    else:
        raise ValueError("DAG workload is defined for single-limb moduli")
    return Dag(seed, p, n_parties, in_width, depth, kind, level, width, src1, off1,
               src2, off2, const)


def triple_array_id(op: int) -> int:
    """Array id of the Beaver triple (a, b, c) consumed by op `op` (+0, +1, +2)."""
    from . import ARR_DAG_TRIPLE0
    return ARR_DAG_TRIPLE0 + 3 * op


OP_TABLE_DTYPE = np.dtype([("kind", np.int32), ("level", np.int32), ("width", np.int64),
                           ("src1", np.int64), ("off1", np.int64), ("src2", np.int64),
                           ("off2", np.int64), ("konst", np.uint64)])


def to_op_table(dag: Dag) -> np.ndarray:
    """The op table in the C layout of spdz_dag_op (smul operand 2 is unused: src2 = 0)."""
    t = np.zeros(dag.n_ops, dtype=OP_TABLE_DTYPE)
    t["kind"] = dag.kind
    t["level"] = dag.level
    t["width"] = dag.width
    t["src1"] = dag.src1
    t["off1"] = dag.off1
    t["src2"] = np.where(dag.src2 >= 0, dag.src2, 0)
    t["off2"] = dag.off2
    t["konst"] = dag.const
    return t

