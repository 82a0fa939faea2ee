"""Pins of the control-flow interpreter (oracle/program.py) on the CPU.

A plaintext evaluation of each program (cleartext field elements, the program's
definition read directly: select as f + c (t - f), shl as a product with 2^k, a
layer as W x + b) must equal the reconstruction of the oracle's shares; MAC
shares must reconstruct to alpha times the value; every opened value must equal
the plaintext value of what was opened; block-entry counts follow the control
flow; secret control flow and malformed programs are rejected.
"""
import numpy as np
import pytest

import oracle.fast as F
from oracle.program import ProgramError, parse, run_program
from workloads import P61, P127, P_PAPER, P_TINY, programs as P


def plain_run(text: str, p: int, seed: int):
    """Cleartext execution: every value a list of integers."""
    prog = parse(text, p)
    f = F.Field(p)
    val, opened, entries = {}, [], 0
    for nid, nd in prog.nodes.items():
        if nd.op == "input":
            val[nid] = [int(v) for v in F.from_limbs(f.deal_values(seed, nd.imm[0], nd.width))]
        elif nd.op == "const":
            val[nid] = nd.imm * nd.width if len(nd.imm) == 1 else list(nd.imm)

    def get(nid, w):
        v = val[nid]
        return v * w if len(v) == 1 and w > 1 else v

    blk, pred = prog.entry, None
    while True:
        entries += 1
        b = prog.blocks[blk]
        at_entry = dict(val)
        for nid in b.lines:
            nd = prog.nodes[nid]
            w = nd.width
            if nd.op == "phi":
                val[nid] = at_entry[[v for v, bb in nd.phi if bb == pred][0]]
            elif nd.op in ("add", "sub", "mul"):
                x, y = get(nd.args[0], w), get(nd.args[1], w)
                op = {"add": lambda a, c: (a + c) % p, "sub": lambda a, c: (a - c) % p,
                      "mul": lambda a, c: (a * c) % p}[nd.op]
                val[nid] = [op(a, c) for a, c in zip(x, y)]
                if nd.op == "mul" and prog.nodes[nd.args[0]].secret and prog.nodes[nd.args[1]].secret:
                    opened.append(None)   # d, e: masked, not comparable in cleartext
            elif nd.op == "lt":
                val[nid] = [int(a < c) for a, c in zip(get(nd.args[0], w), get(nd.args[1], w))]
            elif nd.op == "eq":
                val[nid] = [int(a == c) for a, c in zip(get(nd.args[0], w), get(nd.args[1], w))]
            elif nd.op == "bcast":
                val[nid] = val[nd.args[0]] * nd.imm[0]
            elif nd.op == "cat":
                val[nid] = val[nd.args[0]] + val[nd.args[1]]
            elif nd.op in ("div", "mod"):
                k = nd.imm[0]
                val[nid] = [a // k if nd.op == "div" else a % k for a in val[nd.args[0]]]
            elif nd.op == "reduce":
                val[nid] = [sum(val[nd.args[0]]) % p]
            elif nd.op == "open":
                val[nid] = val[nd.args[0]]
                opened.append(val[nid])
            elif nd.op == "load":
                s = val[nd.args[1]][0]
                val[nid] = val[nd.args[0]][s:s + nd.imm[0]]
            elif nd.op == "layer":
                din, dout, _ = nd.imm
                x, W, bb = (val[i] for i in nd.args)
                val[nid] = [(sum(W[r * din + k] * x[k] for k in range(din)) + bb[r]) % p for r in range(dout)]
                opened.append(None)
        if b.term[0] == "ret":
            break
        if b.term[0] == "br":
            nxt = b.term[1]
        else:
            nxt = b.term[2] if val[b.term[1]][0] != 0 else b.term[3]
        pred, blk = blk, nxt
    return val, [o for o in opened if o is not None], entries


PROGRAMS = [("pipeline", P.pipeline(37)), ("branch", P.branch(21)), ("loop", P.loop(13, 4)),
            ("nested", P.nested(9, 3)), ("select_shl_load", P.select_shl_load(40, 10, 7)),
            ("revealed_branch", P.revealed_branch(11)), ("opened_operand", P.opened_operand(10)),
            ("layer", P.layer(9, 7, 3)), ("layer_public_bias", P.layer_public_bias(9, 7, 3)),
            ("loop_program", P.loop_program(16, 3)), ("one_block_loop", P.one_block_loop(12, 4)),
            ("phi_swap", P.phi_swap(6, 5)), ("public_div_mod", P.public_div_mod(11)),
            ("public_phi_swap", P.public_phi_swap(5, 6)), ("broadcast", P.broadcast(9)),
            ("loop_reads_source", P.loop_reads_source(7, 3)),
            ("lane_constants", P.lane_constants(9)),
            ("concatenation", P.concatenation(5))]


def check_reconstructs(text: str, p: int, n: int, seed: int = 5):
    """The oracle's shares of every output reconstruct to the cleartext run's values (MAC
    shares to alpha times them), every open's plaintext appears in the opened log in order,
    the block-entry counts agree and the MAC check accepts."""
    res = run_program(text, p, n, seed, seed)
    plain, plain_open, entries = plain_run(text, p, seed)
    al = sum(F.from_limbs(res["alpha"].T.copy())) % p
    for o, v in res["outputs"].items():
        want = plain[o]
        if isinstance(v, F.Shares):
            vals = [F.from_limbs(v.val[i]) for i in range(n)]
            macs = [F.from_limbs(v.mac[i]) for i in range(n)]
            got = [sum(q[e] for q in vals) % p for e in range(v.width)]
            gotm = [sum(q[e] for q in macs) % p for e in range(v.width)]
            assert got == want, f"output {o}"
            assert gotm == [al * x % p for x in want], f"output {o} MAC"
        else:
            assert [int(x) for x in F.from_limbs(v)] == want, f"public output {o}"
    opened_pub = [[int(x) for x in F.from_limbs(o)] for o in res["opened"]]
    # the plaintext of every open (the masked d, e and D, E are not comparable) appears in order
    it = iter(opened_pub)
    for want in plain_open:
        assert any(got == want for got in it)
    assert res["entries"] == entries
    assert res["ok"] and sum(int(s) for s in F.from_limbs(res["sigma"].T.copy())) % p == 0


@pytest.mark.parametrize("p,n", [(P_PAPER, 2), (P61, 3), (P_TINY, 2)])
@pytest.mark.parametrize("name,text", PROGRAMS)
def test_program_reconstructs_plaintext(name, text, p, n):
    if name == "revealed_branch" and p == P_TINY:
        pytest.skip("its constant exceeds p = 101")
    check_reconstructs(text, p, n)


@pytest.mark.parametrize("seed", range(160))
def test_random_program_reconstructs_plaintext(seed):
    """Seeded random programs (branches merged by phis mixing public and secret values, loops
    of one block with phis that take each other's values, zero-trip loops, nested regions,
    opens fed back as public operands) over the four fields and widths 1..9."""
    p, n = [(P_PAPER, 2), (P61, 3), (P_TINY, 2), (P127, 2)][seed % 4]
    text = P.random_program(seed, [1, 2, 5, 9][seed // 4 % 4], regions=4 + seed % 5, depth=3 if seed % 3 == 0 else 2)
    check_reconstructs(text, p, n)


def test_loop_closed_form():
    """acc_T = x y^T + sum_{i<T} i y^(T-1-i) for the loop program, in Python integers."""
    p, T, W = P_PAPER, 5, 7
    res = run_program(P.loop(W, T), p, 2, 3, 3)
    f = F.Field(p)
    x = [int(v) for v in F.from_limbs(f.deal_values(3, 0, W))]
    y = [int(v) for v in F.from_limbs(f.deal_values(3, 1, W))]
    want = [(x[e] * pow(y[e], T, p) + sum(i * pow(y[e], T - 1 - i, p) for i in range(T))) % p for e in range(W)]
    assert [int(v) for v in F.from_limbs(res["outputs"][12])] == want
    assert res["entries"] == 1 + (T + 1) + T + 1


@pytest.mark.parametrize("T", [1, 2, 5])
def test_one_block_loop_recurrence(T):
    """The one-block loop against its recurrence in Python integers: phis read the values
    held at the block's entry, so b gets a's previous value (reading a's new value instead,
    or s's before the open, changes the result)."""
    p, W = P_PAPER, 6
    res = run_program(P.one_block_loop(W, T), p, 2, 7, 7)
    f = F.Field(p)
    a = [int(v) for v in F.from_limbs(f.deal_values(7, 0, W))]
    b = [int(v) for v in F.from_limbs(f.deal_values(7, 1, W))]
    s = 0
    for _ in range(T):
        b_entry = b                      # phi 12 at this entry
        a_next = [(a[e] * b[e] + s) % p for e in range(W)]
        a, b, s = a_next, a, sum(a_next) % p
    assert [int(v) for v in F.from_limbs(res["outputs"][20])] == a
    got_b = res["outputs"][12]
    assert [sum(int(got_b.val[i, 0, e]) for i in range(2)) % p for e in range(W)] == b_entry
    assert res["entries"] == 1 + T + 1 and res["ok"]


@pytest.mark.parametrize("T", [1, 2, 7])
def test_public_phi_pair_is_fibonacci(T):
    """u, v = v, u + v through two public phis of one block: at the last entry u = F(T), v = F(T+1);
    s, t = t, s alternate between 0 and T; the secret accumulator follows acc = acc (u + s) + y."""
    p, W = P_PAPER, 4
    res = run_program(P.public_phi_swap(W, T), p, 2, 5, 5)
    fib = [1, 1]
    while len(fib) < T + 3:
        fib.append(fib[-1] + fib[-2])
    u = [int(v) for v in F.from_limbs(res["outputs"][11])]
    v = [int(v) for v in F.from_limbs(res["outputs"][12])]
    assert u == [fib[T - 1]] and v == [fib[T]]
    f = F.Field(p)
    x = [int(a) for a in F.from_limbs(f.deal_values(5, 0, W))]
    y = [int(a) for a in F.from_limbs(f.deal_values(5, 1, W))]
    acc = x
    for k in range(T):
        sk = 0 if k % 2 == 0 else T
        acc = [(a * (fib[k] + sk) + b) % p for a, b in zip(acc, y)]
    assert [int(a) for a in F.from_limbs(res["outputs"][16])] == acc
    assert [int(a) for a in F.from_limbs(res["outputs"][20])] == [0 if (T - 1) % 2 == 0 else T]


@pytest.mark.parametrize("T", [1, 2, 3, 6])
def test_phi_swap_exchanges(T):
    """Two phis reading each other exchange their values on every back edge."""
    p, W = P61, 5
    res = run_program(P.phi_swap(W, T), p, 2, 2, 2)
    f = F.Field(p)
    x = [int(v) for v in F.from_limbs(f.deal_values(2, 0, W))]
    y = [int(v) for v in F.from_limbs(f.deal_values(2, 1, W))]
    a = x if (T - 1) % 2 == 0 else y
    got = res["outputs"][11]
    assert [sum(int(got.val[i, 0, e]) for i in range(2)) % p for e in range(W)] == a
    assert [int(v) for v in F.from_limbs(res["outputs"][15])] == [x[e] * y[e] % p for e in range(W)]


@pytest.mark.parametrize("p", [P_PAPER, P61, P127])
def test_div_mod_of_public_values(p):
    """div and mod take a public value as an integer in [0, p): checked on constants whose
    quotients and remainders are known, and on a dealt public vector against Python's // and %."""
    text = """
input 1 public 9 0
const 2 1 4001
const 3 1 100
output 4
output 5
output 6
output 7
block 0
4 = mod 1 4001
5 = div 1 32
6 = mod 2 32
7 = div 3 7
ret
"""
    res = run_program(text, p, 2, 3, 3)
    v = [int(a) for a in F.from_limbs(F.Field(p).deal_values(3, 0, 9))]
    out = {o: [int(a) for a in F.from_limbs(res["outputs"][o])] for o in (4, 5, 6, 7)}
    assert out[4] == [a % 4001 for a in v] and out[5] == [a // 32 for a in v]
    assert out[6] == [4001 % 32] == [1] and out[7] == [14]
    with pytest.raises(ProgramError, match="secret"):
        parse("input 1 private 4 0\nblock 0\n2 = div 1 4\nret\n", p)
    with pytest.raises(ProgramError):
        parse("input 1 public 4 0\nblock 0\n2 = mod 1 0\nret\n", p)


def test_nested_entries_follow_the_inner_trip_counts():
    outer = 4
    res = run_program(P.nested(3, outer), P61, 2, 1, 1)
    inner = sum(i + 1 for i in range(outer))
    # entry + outer headers + outer bodies + inner headers + inner bodies + latches + exit
    assert res["entries"] == 1 + (outer + 1) + outer + (inner + outer) + inner + outer + 1


def test_secret_control_flow_rejected():
    with pytest.raises(ProgramError):
        parse(P.secret_branch(4), P_PAPER)


@pytest.mark.parametrize("bad", [
    "input 1 private 4 0\ninput 2 private 5 1\nblock 0\n3 = add 1 2\nret\n",        # widths
    "input 1 private 4 0\nblock 0\n2 = lt 1 1\nret\n",                                # secret comparison
    "input 1 public 4 0\nblock 0\n2 = open 1\nret\n",                                 # open of a public value
    "const 1 1 200\nblock 0\nret\n",                                                  # constant not below p
])
def test_malformed_programs_rejected(bad):
    with pytest.raises(ProgramError):
        parse(bad, P_TINY)


def test_mac_log_order_is_program_order():
    """The first opened values of the pipeline program are the product's d and e, then w, then s."""
    p, W = P_PAPER, 12
    res = run_program(P.pipeline(W), p, 2, 7, 7)
    assert [o.shape[1] for o in res["opened"]] == [W, W, W, 1]
    plain, plain_open, _ = plain_run(P.pipeline(W), p, 7)
    assert [int(v) for v in F.from_limbs(res["opened"][2])] == plain[7]
    assert [int(v) for v in F.from_limbs(res["opened"][3])] == plain[8]
