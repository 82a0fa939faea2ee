"""Seeded synthetic workloads for the SPDZ online-phase hot path.

This module is shared by the oracle, the tests and the benchmark.  It only
*describes* inputs: field moduli, party counts, sizes, seeds, the stream-id
layout that the dealers (fake preprocessing) key their counter-based
generator on, and the structure of the layered DAG workload.  It contains
none of the protocol's modular arithmetic: dealing shares, MACs and triples
is done separately by the oracle (on the CPU) and by the device library.

Stream-id layout (both dealers derive every random word from it):

    stream(tag, array_id, party) = tag << 56 | array_id << 8 | party

    TAG_ALPHA  party i's MAC-key share alpha_i is element i of stream(TAG_ALPHA, 0, 0)
    TAG_VALUE  element e of the secret held in array k
    TAG_SHARE  value share of party i < n-1 for array k (party n-1 takes the remainder)
    TAG_MACSH  MAC share of party i < n-1 for array k (party n-1 takes the remainder)
    TAG_COEF   MAC-check coefficient r_j of check number `epoch` (array_id = epoch)

The generator itself (SplitMix64 used in counter mode, plus rejection
sampling into [0, p)) is specified in the oracle and in the device header.
"""
from __future__ import annotations

from dataclasses import dataclass

P61 = (1 << 61) - 1
P127 = (1 << 127) - 1
P_PAPER = (1 << 32) - 5  # field of the paper's evaluation (Sec. IV-A)
P_TINY = 101             # brute-force field for exhaustive tests

TAG_ALPHA = 1
TAG_VALUE = 2
TAG_SHARE = 3
TAG_MACSH = 4
TAG_COEF = 5

# array ids of the element-wise workloads
ARR_X, ARR_Y, ARR_A, ARR_B, ARR_C = 0, 1, 2, 3, 4
# matrix-triple workload: X, Y, then triple (A, B, C)
ARR_MX, ARR_MY, ARR_MA, ARR_MB, ARR_MC = 8, 9, 10, 11, 12
# DAG workload: the two level-0 inputs, then 3 ids (a, b, c) per Beaver op
ARR_DAG_IN0, ARR_DAG_IN1 = 16, 17
ARR_DAG_TRIPLE0 = 32
# linear-layer workload: W, x, b, then the matrix-vector triples (A, B, C)
ARR_LW, ARR_LX, ARR_LB, ARR_LA, ARR_LB_T, ARR_LC = 20, 21, 22, 23, 24, 25

SEED_PARITY = 0
SEEDS_TIMING = (1, 2, 3, 4, 5)
SEEDS_TRAIN = tuple(range(100, 200))
SEEDS_HELDOUT = tuple(range(1000, 1020))


def stream_id(tag: int, array_id: int, party: int = 0) -> int:
    assert 0 <= tag < 256 and 0 <= array_id < (1 << 48) and 0 <= party < 256
    return (tag << 56) | (array_id << 8) | party


def n_limbs(p: int) -> int:
    """64-bit limbs per residue: 1 for p < 2^64, 2 for p < 2^127."""
    assert p > 2 and p % 2 == 1
    if p < (1 << 64):
        return 1
    assert p < (1 << 127)
    return 2


@dataclass(frozen=True)
class ElementwiseConfig:
    name: str
    n: int          # simulated parties
    p: int          # prime modulus
    width: int      # elements per batch
    fused_linear: bool  # C1-style pipeline: w = z + 3x - y, s = sum z, opens w and s
    seed: int = SEED_PARITY

    @property
    def L(self) -> int:
        return n_limbs(self.p)


# The two element-wise workloads: plain Beaver at 2 parties over 2^61-1, and
# Beaver + fused linear op + secret dot product at 3 parties over 2^127-1.
BEAVER_P61 = ElementwiseConfig("beaver_n2_p61_w65536", 2, P61, 1 << 16, False)
PIPELINE_P127 = ElementwiseConfig("beaver_linear_dot_n3_p127_w16777216", 3, P127, 1 << 24, True)

# Coefficients of the fused linear op w = 1*z + 3*x + (p-1)*y (i.e. z + 3x - y).
def pipeline_coeffs(p: int):
    return (1, 3, p - 1)


@dataclass(frozen=True)
class MatmulConfig:
    name: str
    n: int
    p: int
    N: int
    seed: int = SEED_PARITY


MATMUL_1024 = MatmulConfig("matrix_triple_n2_p61_N1024", 2, P61, 1024)
MATMUL_4096 = MatmulConfig("matrix_triple_n2_p61_N4096", 2, P61, 4096)


@dataclass(frozen=True)
class LayerConfig:
    """The paper's private linear layer y = W x + b (Sec. III-D, IV-A): W is dout x din,
    row-major; W is cut into tiles of `tile_rows` consecutive rows, tile_rows =
    max(1, slice // din) for a slice size counted in elements of W."""
    name: str
    n: int
    p: int
    din: int
    dout: int
    slice: int
    seed: int = SEED_PARITY

    @property
    def tile_rows(self) -> int:
        return max(1, self.slice // self.din)

    @property
    def n_tiles(self) -> int:
        return -(-self.dout // self.tile_rows)


def layer_config(dim: int, slice_size: int = 524280, n: int = 2) -> LayerConfig:
    return LayerConfig(f"linear_layer_n{n}_p32_d{dim}_s{slice_size}", n, P_PAPER, dim, dim, slice_size)


# the paper's input-size sweep (Sec. IV-E: 2 parties, slice 524280) and slice sweep at 8192 (Sec. IV-D)
LAYER_DIMS = (2048, 4096, 8192)
LAYER_SLICES = (131070, 262140, 524280, 1048560)


def tamper_index(seed: int, width: int) -> int:
    """Element whose last-party value share is bumped by one in the rejection run."""
    import numpy as np
    return int(np.random.default_rng([seed, 0x7A3]).integers(0, width))
