"""Programs for the control-flow runtime: a data-flow graph per basic block plus
the control-flow graph between blocks, as a compiler front end would emit them
(Sec. III-B, "Compile-time Control-Flow Analysis").  This module holds the text
format's definition and seeded example programs; it contains no arithmetic.

Text format (one statement per line, '#' starts a comment, ids are integers):

    input <id> private|public <width> <array_id>
        secret input dealt from array <array_id>, or public input whose values are
        element 0..width-1 of that array's value stream
    const <id> <width> <value>          public vector, every entry <value> (0 <= value < p)
    const <id> <width> <v0> ... <v(w-1)>  public vector, one value per lane
    output <id>                         a result: the value of <id> when the program returns
    block <bid>                         the following lines belong to block <bid>; the first
                                        block of the file is the entry
    <id> = add|sub|mul <a> <b>          widths equal, or one operand a public scalar
    <id> = shl <a> <k>                  a * 2^k, k a literal (lowered, see below)
    <id> = select <c> <t> <f>           f + c (t - f) (lowered, see below)
    <id> = lt|eq <a> <b>                public operands only: 1 if a < b (a = b) as integers
    <id> = div|mod <a> <k>              public a only, k a literal >= 1: each element of a,
                                        an integer in [0, p), divided by k (quotient or
                                        remainder; loop-count arithmetic such as a bound
                                        rounded down to a multiple of the vector length)
    <id> = bcast <a> <w>                a value of width 1 (secret or public) repeated w times
    <id> = cat <a> <b>                  the lanes of a followed by those of b (a public one shared
                                        when the other is secret)
    <id> = reduce <a>                   sum of the elements (width 1)
    <id> = open <a>                     reveal a secret value (public result)
    <id> = load <base> <start> <count>  elements start .. start+count-1 of base; <start> is a
                                        public scalar node
    <id> = phi <v1> <b1> [<v2> <b2> ...]  value vk when the block was entered from block bk:
                                        vk as it was at that entry, also where vk is a node
                                        of the block itself (a loop of one block) or another
                                        phi of it (the phis of a block read their values
                                        all at once, as LLVM's do)
    <id> = layer <x> <W> <b> <din> <dout> <tile_rows>   linear layer W x + b, x and W
                                        secret; b secret or public (a public b enters as
                                        a public constant: party 0 adds it, every MAC
                                        share alpha_i b)
    br <bid>                            terminators: one per block, last line of the block
    cbr <cond> <bid_true> <bid_false>   cond a public scalar; nonzero selects bid_true
    ret

A value is secret if it depends on a private input (secret inputs, and any op with a
secret operand); lt/eq take public operands and open takes a secret one; a conditional
branch on a secret condition is rejected (control flow must be public).  Source ids are
below 2^14.  Lowering, part of the format's meaning (both executors apply it):
  select(c, t, f) at id v:  v + 2^14 = sub t f;  v + 2 * 2^14 = mul c (v + 2^14);
                            v = add f (v + 2 * 2^14)
  shl(a, k) at id v:        v + 2^14 = const 1 (2^k mod p);  v = mul a (v + 2^14)
in that order, in place of the original line.

Semantics: blocks execute one at a time in control-flow order, the lines of a block in
order; every line of an entered block executes once per entry.  The opened-value log
records, in this order, each secret-by-secret product's d then e, each open's values,
and each layer's D_t then E_t per tile.  The k-th execution of product node v (k = 0, 1,
...) consumes the Beaver triple dealt as arrays PROG_TRIPLE0 + 3 (v + 2^16 k) (+0 a, +1 b,
+2 c); the k-th execution of layer node v the matrix-vector triples dealt from array
PROG_TRIPLE0 + 3 (v + 2^16 k).
"""
from __future__ import annotations

PROG_TRIPLE0 = 1 << 20
AUX = 1 << 14
NODE_STRIDE = 1 << 16
MAX_BLOCK_ENTRIES = 1_000_000


def triple_array(node: int, instance: int) -> int:
    return PROG_TRIPLE0 + 3 * (node + NODE_STRIDE * instance)


def pipeline(W: int) -> str:
    """z = x y, w = z + 3x - y, s = sum z, open w and s (straight-line)."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 1 3
output 4
output 9
output 10
block 0
4 = mul 1 2
5 = mul 1 3
6 = sub 4 2
7 = add 6 5
8 = reduce 4
9 = open 7
10 = open 8
ret
"""


def branch(W: int, t_array: int = 2) -> str:
    """if t < 5 (public t): r = x y else r = x + y; r merged by a phi and opened."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
input 3 public 1 {t_array}
const 4 1 5
output 8
output 9
block 0
5 = lt 3 4
cbr 5 1 2
block 1
6 = mul 1 2
br 3
block 2
7 = add 1 2
br 3
block 3
8 = phi 6 1 7 2
9 = open 8
ret
"""


def loop(W: int, trips: int) -> str:
    """acc = x; for i in 0 .. trips-1: acc = acc y + i; open acc."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 1 {trips}
const 4 1 0
const 5 1 1
output 6
output 12
block 0
br 1
block 1
6 = phi 1 0 9 2
7 = phi 4 0 10 2
8 = lt 7 3
cbr 8 2 3
block 2
11 = mul 6 2
9 = add 11 7
10 = add 7 5
br 1
block 3
12 = open 6
ret
"""


def one_block_loop(W: int, trips: int) -> str:
    """A loop whose body is one block branching back to itself (the shape clang -O2 gives a
    counted loop): a, b, s = x, y, 0, then trips times a, b, s = a b + s, a, sum(a b + s),
    the sum opened each trip.  b's phi reads a's phi (its value at the entry), s's phi the
    open of the previous trip; the final a is opened."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 1 {trips}
const 4 1 0
const 5 1 1
output 12
output 20
block 0
br 1
block 1
10 = phi 4 0 17 1
11 = phi 1 0 14 1
12 = phi 2 0 11 1
13 = phi 4 0 16 1
18 = mul 11 12
14 = add 18 13
15 = reduce 14
16 = open 15
17 = add 10 5
19 = lt 17 3
cbr 19 1 2
block 2
20 = open 14
ret
"""


def phi_swap(W: int, trips: int) -> str:
    """a, b = x, y, then trips - 1 times a, b = b, a in a one-block loop: two phis that read
    each other; a b opened at the end."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 1 {trips}
const 4 1 0
const 5 1 1
output 11
output 15
block 0
br 1
block 1
10 = phi 4 0 13 1
11 = phi 1 0 12 1
12 = phi 2 0 11 1
13 = add 10 5
14 = lt 13 3
cbr 14 1 2
block 2
16 = mul 11 12
15 = open 16
ret
"""


def public_div_mod(W: int) -> str:
    """Integer quotient and remainder of a public vector by literals, one of them scaling a
    secret vector that is then opened."""
    return f"""
input 1 public {W} 0
input 2 private {W} 1
output 3
output 4
output 6
block 0
3 = mod 1 4001
4 = div 1 32
5 = mul 2 3
6 = open 5
ret
"""


def public_phi_swap(W: int, trips: int) -> str:
    """Public phis of one block that read each other: u, v = v, u + v (a Fibonacci pair) and a
    swapped pair s, t = t, s starting at 0, trips; a secret accumulator scaled by u + s on every
    trip: acc = x, then acc = acc (u + s) + y."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 1 {trips}
const 4 1 0
const 5 1 1
output 11
output 12
output 13
output 16
output 20
block 0
br 1
block 1
10 = phi 4 0 14 1
11 = phi 5 0 12 1
12 = phi 5 0 15 1
13 = phi 1 0 18 1
20 = phi 4 0 21 1
21 = phi 3 0 20 1
22 = add 11 20
17 = mul 13 22
18 = add 17 2
15 = add 11 12
14 = add 10 5
19 = lt 14 3
cbr 19 1 2
block 2
16 = open 18
ret
"""


def broadcast(W: int) -> str:
    """A secret and a public scalar repeated across W lanes: z = bcast(s) y + bcast(c), opened."""
    return f"""
input 1 private 1 0
input 2 private {W} 1
input 3 public 1 2
output 6
output 8
block 0
4 = bcast 1 {W}
5 = bcast 3 {W}
7 = mul 4 2
6 = add 7 5
8 = open 6
ret
"""


def loop_reads_source(W: int, trips: int) -> str:
    """The loop program with its back-edge value also read after the loop: acc = x; for i <
    trips: v = acc y + i, acc = v; then open acc and v - acc (zero) and output v."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 1 {trips}
const 4 1 0
const 5 1 1
output 9
output 12
output 14
block 0
br 1
block 1
6 = phi 1 0 9 2
7 = phi 4 0 10 2
8 = lt 7 3
cbr 8 2 3
block 2
11 = mul 6 2
9 = add 11 7
10 = add 7 5
br 1
block 3
12 = open 6
13 = sub 9 6
14 = open 13
ret
"""


def nested(W: int, outer: int) -> str:
    """for i < outer: for j < i + 1: acc = acc * y + x; acc opened after every outer
    iteration (its reduction); the inner trip count depends on the outer counter."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 1 {outer}
const 4 1 0
const 5 1 1
output 20
output 31
block 0
br 1
block 1
20 = phi 1 0 24 4
21 = phi 4 0 27 4
22 = lt 21 3
cbr 22 2 5
block 2
27 = add 21 5
br 3
block 3
23 = phi 20 2 25 6
26 = phi 4 2 28 6
29 = lt 26 27
cbr 29 6 4
block 6
30 = mul 23 2
25 = add 30 1
28 = add 26 5
br 3
block 4
24 = add 23 4
32 = reduce 24
33 = open 32
br 1
block 5
31 = open 20
ret
"""


def select_shl_load(W: int, count: int, start: int) -> str:
    """r = select(c, x, y) with a secret c; s = shl(r, 5); v = load(s, start, count)
    with a public start computed from constants; u = v * open(reduce(v)) (public scalar)."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
input 3 private {W} 2
const 4 1 {start - 1}
const 5 1 1
output 7
output 10
output 12
block 0
6 = select 3 1 2
7 = shl 6 5
8 = add 4 5
10 = load 7 8 {count}
11 = reduce 10
13 = open 11
12 = mul 10 13
ret
"""


def revealed_branch(W: int) -> str:
    """b = open(reduce(x y)); if b < p/2: out = x y - x else out = x y + y (a branch on a
    revealed value), then one more product of the result with x."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 1 2147483646
output 9
output 10
block 0
4 = mul 1 2
5 = reduce 4
6 = open 5
7 = lt 6 3
cbr 7 1 2
block 1
8 = sub 4 1
br 3
block 2
11 = add 4 2
br 3
block 3
12 = phi 8 1 11 2
9 = mul 12 1
10 = open 9
ret
"""


def opened_operand(W: int) -> str:
    """Secret and public operands where the public one was opened just before:
    r = x - open(reduce(x)), q = open(reduce(y)) - y, u = r q, opened (the opened
    value is read by the next node while its host copy may still be in flight)."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
output 5
output 8
output 10
block 0
3 = reduce 1
4 = open 3
5 = sub 1 4
6 = reduce 2
7 = open 6
8 = sub 7 2
9 = mul 5 8
10 = open 9
ret
"""


def layer(din: int, dout: int, tile_rows: int) -> str:
    """y = W x + b (private linear layer), then z = y y opened."""
    return f"""
input 1 private {din} 0
input 2 private {din * dout} 1
input 3 private {dout} 2
output 4
output 6
block 0
4 = layer 1 2 3 {din} {dout} {tile_rows}
5 = mul 4 4
6 = open 5
ret
"""


def layer_public_bias(din: int, dout: int, tile_rows: int) -> str:
    """y = W x + b with a public bias b (the paper's Fig. 2 annotations), y opened."""
    return f"""
input 1 private {din} 0
input 2 private {din * dout} 1
input 3 public {dout} 2
output 4
output 5
block 0
4 = layer 1 2 3 {din} {dout} {tile_rows}
5 = open 4
ret
"""


def secret_branch(W: int) -> str:
    """A conditional branch on a secret value: must be rejected."""
    return f"""
input 1 private 1 0
input 2 private {W} 1
block 0
cbr 1 1 2
block 1
3 = mul 2 2
br 2
block 2
ret
"""


def loop_program(W: int, trips: int) -> str:
    """The runtime's measured program: a loop whose body holds a batch of independent
    products and additions of width W (an inner product pipeline over `trips` rounds):
    acc <- acc * y + x; t <- acc * x; u <- t + y, then one open at the end."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 1 {trips}
const 4 1 0
const 5 1 1
output 6
output 15
block 0
br 1
block 1
6 = phi 1 0 9 2
7 = phi 4 0 10 2
8 = lt 7 3
cbr 8 2 3
block 2
11 = mul 6 2
9 = add 11 1
12 = mul 9 1
13 = add 12 2
14 = mul 13 6
10 = add 7 5
br 1
block 3
16 = reduce 6
15 = open 16
ret
"""


def random_program(seed: int, W: int, regions: int = 5, depth: int = 2) -> str:
    """A seeded random program over vectors of width W: straight runs of +, -, * (secret by
    secret, by a public vector, by a public scalar), shl, select, opens whose values come back
    as public operands, secret or public sums broadcast back to W lanes, public div / mod;
    public branches (on a public input or on an opened sum's parity) merged by phis that may
    mix a public and a secret value; loops of one block (counter, carried phis, sometimes two
    phis that take each other's values, body values read after the loop) and of a header and
    a body (0..3 trips, nested regions in the body).  Every loop has a literal trip count, so
    every program ends; constants stay below 101, so every field of the format accepts them."""
    import random
    rng = random.Random(seed)
    head, order, body = [], [], {}
    ids = [0]
    consts = {}
    cur = [0]
    secret = {}

    def new():
        ids[0] += 1
        return ids[0]

    def const(v):
        if v not in consts:
            c = new()
            consts[v] = c
            head.append(f"const {c} 1 {v}")
        return consts[v]

    def start(b):
        cur[0] = b
        body[b] = []
        order.append(b)

    def emit(line):
        body[cur[0]].append(line)

    nblk = [1]

    def newblock():
        nblk[0] += 1
        return nblk[0] - 1

    xs = [new() for _ in range(3)]
    for k, v in enumerate(xs):
        head.append(f"input {v} private {W} {k}")
        secret[v] = True
    pv = new()
    head.append(f"input {pv} public {W} 3")
    secret[pv] = False
    ps = new()
    head.append(f"input {ps} public 1 4")

    def put(v, is_secret, S, P):
        secret[v] = is_secret
        (S if is_secret else P).append(v)
        return v

    def elementwise(S, P, out=None, a=None):
        """one secret result of width W, written to `out` if given; `a`, the secret operand,
        drawn from S if not given"""
        v = new() if out is None else out
        a = rng.choice(S) if a is None else a
        r = rng.random()
        if r < 0.28:
            emit(f"{v} = mul {a} {rng.choice(S)}")
        elif r < 0.38:
            emit(f"{v} = mul {rng.choice(P)} {a}")
        elif r < 0.46:
            emit(f"{v} = mul {a} {const(rng.randrange(2, 100))}")
        elif r < 0.64:
            emit(f"{v} = add {a} {rng.choice(S + P)}")
        elif r < 0.80:
            b = rng.choice(S + P)
            emit(f"{v} = sub {b} {a}" if rng.random() < 0.5 else f"{v} = sub {a} {b}")
        elif r < 0.86:
            emit(f"{v} = add {rng.choice([ps, const(rng.randrange(0, 100))])} {a}")
        elif r < 0.93:
            emit(f"{v} = shl {a} {rng.randrange(0, 40)}")
        else:
            emit(f"{v} = select {rng.choice(S + P)} {a} {rng.choice(S + P)}")
        secret[v] = True
        return v

    def straight(S, P, k):
        for _ in range(k):
            r = rng.random()
            if r < 0.08:
                put(new(), False, S, P)
                emit(f"{P[-1]} = open {rng.choice(S)}")
            elif r < 0.14:
                src = rng.choice(S + P)
                s, b = new(), new()
                emit(f"{s} = reduce {src}")
                emit(f"{b} = bcast {s} {W}")
                put(b, secret[src], S, P)
            elif r < 0.20:
                q = new()
                emit(f"{q} = {rng.choice(['add', 'mul', 'sub'])} {rng.choice(P)} {rng.choice(P)}")
                put(q, False, S, P)
            elif r < 0.24:
                q = new()
                emit(f"{q} = {rng.choice(['div', 'mod'])} {rng.choice(P)} {rng.randrange(1, 9)}")
                put(q, False, S, P)
            else:
                S.append(elementwise(S, P))

    def branch_region(S, P, d):
        if rng.random() < 0.5:
            c = new()
            emit(f"{c} = lt {ps} {const(rng.randrange(0, 100))}")
        else:
            s, o, c = new(), new(), new()
            emit(f"{s} = reduce {rng.choice(S)}")
            emit(f"{o} = open {s}")
            emit(f"{c} = mod {o} 2")
        T, Fb, M = newblock(), newblock(), newblock()
        emit(f"cbr {c} {T} {Fb}")
        sides = []
        for b in (T, Fb):
            start(b)
            S2, P2 = list(S), list(P)
            region_seq(S2, P2, d - 1, rng.randint(0, 2))
            sides.append((cur[0], S2, P2))
            emit(f"br {M}")
        start(M)
        (bt, St, Pt), (bf, Sf, Pf) = sides
        for _ in range(rng.randint(1, 3)):
            vt, vf = rng.choice(St + Pt), rng.choice(Sf + Pf)
            ph = new()
            emit(f"{ph} = phi {vt} {bt} {vf} {bf}")
            put(ph, secret[vt] or secret[vf], S, P)

    def one_block_loop(S, P):
        pre, L, X = cur[0], newblock(), newblock()
        emit(f"br {L}")
        start(L)
        trips = rng.randint(1, 4)
        i, inx = new(), new()
        k = rng.randint(1, 3)
        phis = [new() for _ in range(k)]
        inits = [rng.choice(S + P) for _ in range(k)]
        swap = k >= 2 and rng.random() < 0.4
        nexts = [new() for _ in range(k)]
        if swap:
            nexts[0], nexts[1] = phis[1], phis[0]
        emit(f"{i} = phi {const(0)} {pre} {inx} {L}")
        base = list(S)  # secret whatever the loop's phis turn out to be
        for ph, ini, nx in zip(phis, inits, nexts):
            emit(f"{ph} = phi {ini} {pre} {nx} {L}")
        for j, ph in enumerate(phis):
            if swap and j < 2:
                put(ph, secret[inits[0]] or secret[inits[1]], S, P)
            else:
                put(ph, True, S, P)
        if not S:
            S.append(xs[0])
        straight(S, P, rng.randint(0, 3))
        for j, nx in enumerate(nexts):
            if not (swap and j < 2):
                S.append(elementwise(S, P, out=nx, a=rng.choice(base)))
        c = new()
        emit(f"{inx} = add {i} {const(1)}")
        emit(f"{c} = lt {inx} {const(trips)}")
        emit(f"cbr {c} {L} {X}")
        start(X)

    def header_loop(S, P, d):
        pre, H, B, X = cur[0], newblock(), newblock(), newblock()
        emit(f"br {H}")
        start(H)
        hlines = body[H]
        trips = rng.randint(0, 3)
        i, inx = new(), new()
        k = rng.randint(1, 3)
        phis = [new() for _ in range(k)]
        inits = [rng.choice(S + P) for _ in range(k)]
        nexts = [new() for _ in range(k)]
        c = new()
        start(B)
        base = list(S)
        S2, P2 = list(S), list(P)
        for ph in phis:
            put(ph, True, S2, P2)
        region_seq(S2, P2, d - 1, rng.randint(1, 2))
        for nx in nexts:
            S2.append(elementwise(S2, P2, out=nx, a=rng.choice(base)))
        emit(f"{inx} = add {i} {const(1)}")
        emit(f"br {H}")
        back = cur[0]
        hlines.append(f"{i} = phi {const(0)} {pre} {inx} {back}")
        for ph, ini, nx in zip(phis, inits, nexts):
            hlines.append(f"{ph} = phi {ini} {pre} {nx} {back}")
        hlines.append(f"{c} = lt {i} {const(trips)}")
        hlines.append(f"cbr {c} {B} {X}")
        for ph in phis:
            put(ph, True, S, P)
        start(X)

    def region_seq(S, P, d, count):
        for _ in range(count):
            r = rng.random()
            if d > 0 and r < 0.25:
                branch_region(S, P, d)
            elif d > 0 and r < 0.45:
                one_block_loop(S, P)
            elif d > 0 and r < 0.6:
                header_loop(S, P, d)
            else:
                straight(S, P, rng.randint(1, 4))

    start(0)
    S, P = list(xs), [pv]
    region_seq(S, P, depth, regions)
    outs = rng.sample(S, min(3, len(S))) + rng.sample(P, min(1, len(P)))
    emit("ret")
    head += [f"output {o}" for o in dict.fromkeys(outs)]
    lines = head[:]
    for b in order:
        lines.append(f"block {b}")
        lines += body[b]
    return "\n".join(lines) + "\n"


def lane_constants(W: int) -> str:
    """Public constants with one value per lane: z = x * c + d, opened, and the sum of c x."""
    c = " ".join(str((7 * k + 3) % 100) for k in range(W))
    d = " ".join(str((k * k) % 97) for k in range(W))
    return f"""
input 1 private {W} 0
const 2 {W} {c}
const 3 {W} {d}
output 6
output 8
block 0
4 = mul 1 2
5 = add 4 3
6 = open 5
7 = reduce 4
8 = open 7
ret
"""


def concatenation(W: int) -> str:
    """Lanes joined (W >= 3): cat(x, c) * cat(y, c) with a public constant c of 3 lanes (shared
    into the secret result), a view of it, cat(open(x), c) + a view of cat(x, y), and
    cat(open(x), y); all opened."""
    return f"""
input 1 private {W} 0
input 2 private {W} 1
const 3 3 5 6 7
const 15 1 2
const 17 1 0
output 7
output 10
output 19
block 0
4 = cat 1 3
5 = cat 2 3
6 = mul 4 5
11 = load 6 15 {W}
7 = open 11
8 = open 1
9 = cat 8 3
12 = cat 1 2
13 = load 12 17 {W + 3}
14 = add 9 13
10 = open 14
18 = cat 8 2
19 = open 18
ret
"""
