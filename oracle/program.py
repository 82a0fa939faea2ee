"""Sequential interpreter of control-flow programs -- TEST INFRASTRUCTURE ONLY.

Executes a program in the text format of workloads.programs the plain way: blocks one
at a time in control-flow order (Sec. III-C: control transfers only through branches,
conditions public), the lines of each entered block in order, every secret operation
with the tier-1 oracle's share arithmetic.  Opened values enter one MAC log in that
order; the result is compared bit for bit with the library's non-blocking runtime.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import fast as F
from workloads.programs import AUX, MAX_BLOCK_ENTRIES, triple_array


class ProgramError(Exception):
    pass


@dataclass
class Node:
    id: int
    op: str
    args: List[int] = field(default_factory=list)
    width: int = 1
    secret: bool = False
    block: int = -1
    imm: List[int] = field(default_factory=list)     # literals (shl k, load count, layer dims)
    phi: List[Tuple[int, int]] = field(default_factory=list)


@dataclass
class Block:
    id: int
    lines: List[int] = field(default_factory=list)    # node ids in execution order (after lowering)
    term: Tuple = ("ret",)


@dataclass
class Program:
    nodes: Dict[int, Node]
    blocks: Dict[int, Block]
    entry: int
    outputs: List[int]


def parse(text: str, p: int) -> Program:
    nodes: Dict[int, Node] = {}
    blocks: Dict[int, Block] = {}
    order: List[int] = []
    outputs: List[int] = []
    cur: Optional[Block] = None
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        t = line.split()
        if t[0] == "input":
            nid, kind, w, aid = int(t[1]), t[2], int(t[3]), int(t[4])
            nodes[nid] = Node(nid, "input", [], w, kind == "private", -1, [aid])
        elif t[0] == "const":   # one value for every lane, or one value per lane
            nid, w, vals = int(t[1]), int(t[2]), [int(x) for x in t[3:]]
            if len(vals) != 1 and len(vals) != w:
                raise ProgramError(f"bad line: {raw}")
            for v in vals:
                if not 0 <= v < p:
                    raise ProgramError(f"constant {v} not below p")
            nodes[nid] = Node(nid, "const", [], w, False, -1, vals)
        elif t[0] == "output":
            outputs.append(int(t[1]))
        elif t[0] == "block":
            cur = Block(int(t[1]))
            blocks[cur.id] = cur
            order.append(cur.id)
        elif t[0] == "br":
            cur.term = ("br", int(t[1]))
        elif t[0] == "cbr":
            cur.term = ("cbr", int(t[1]), int(t[2]), int(t[3]))
        elif t[0] == "ret":
            cur.term = ("ret",)
        else:
            if len(t) < 3 or t[1] != "=":
                raise ProgramError(f"bad line: {raw}")
            nid, op, rest = int(t[0]), t[2], [int(v) for v in t[3:]]
            if nid >= AUX:
                raise ProgramError("source ids must be below 2^14")
            lower(nodes, cur, nid, op, rest, p)
    if not order:
        raise ProgramError("no blocks")
    prog = Program(nodes, blocks, order[0], outputs)
    infer(prog)
    return prog


def lower(nodes, blk: Block, nid: int, op: str, a: List[int], p: int):
    def add(n: Node):
        n.block = blk.id
        nodes[n.id] = n
        blk.lines.append(n.id)

    if op == "select":
        c, t, f = a
        add(Node(nid + AUX, "sub", [t, f]))
        add(Node(nid + 2 * AUX, "mul", [c, nid + AUX]))
        add(Node(nid, "add", [f, nid + 2 * AUX]))
    elif op == "shl":
        x, k = a
        nodes[nid + AUX] = Node(nid + AUX, "const", [], 1, False, -1, [pow(2, k, p)])
        add(Node(nid, "mul", [x, nid + AUX]))
    elif op == "load":
        add(Node(nid, "load", [a[0], a[1]], imm=[a[2]]))
    elif op == "phi":
        add(Node(nid, "phi", phi=[(a[i], a[i + 1]) for i in range(0, len(a), 2)]))
    elif op == "layer":
        add(Node(nid, "layer", a[:3], imm=a[3:6]))
    elif op == "bcast":
        if len(a) != 2 or a[1] < 1:
            raise ProgramError("bcast a w with a literal w >= 1")
        add(Node(nid, op, a[:1], imm=[a[1]]))
    elif op in ("div", "mod"):
        if len(a) != 2 or a[1] < 1:
            raise ProgramError(f"{op} a k with a literal k >= 1")
        add(Node(nid, op, a[:1], imm=[a[1]]))
    elif op in ("add", "sub", "mul", "lt", "eq", "cat"):
        add(Node(nid, op, a[:2]))
    elif op in ("reduce", "open"):
        add(Node(nid, op, a[:1]))
    else:
        raise ProgramError(f"unknown op {op}")


def infer(prog: Program):
    """Widths and privacy in definition order (blocks in file order; phi operands may be
    defined later, so phis are settled by iterating to a fixed point)."""
    nodes = prog.nodes
    lines = [nid for b in prog.blocks.values() for nid in b.lines]
    for _ in range(4):
        for nid in lines:
            n = nodes[nid]
            if n.op == "phi":
                ins = [nodes[v] for v, _ in n.phi if v in nodes]
                n.width = max(x.width for x in ins)
                n.secret = any(x.secret for x in ins)
            elif n.op in ("add", "sub", "mul"):
                x, y = nodes[n.args[0]], nodes[n.args[1]]
                n.width = max(x.width, y.width)
                n.secret = x.secret or y.secret
            elif n.op in ("lt", "eq"):
                n.width = max(nodes[n.args[0]].width, nodes[n.args[1]].width)
                n.secret = False
            elif n.op in ("div", "mod"):
                n.width, n.secret = nodes[n.args[0]].width, False
            elif n.op == "cat":
                x, y = nodes[n.args[0]], nodes[n.args[1]]
                n.width, n.secret = x.width + y.width, x.secret or y.secret
            elif n.op == "bcast":
                n.width, n.secret = n.imm[0], nodes[n.args[0]].secret
            elif n.op == "reduce":
                n.width, n.secret = 1, nodes[n.args[0]].secret
            elif n.op == "open":
                n.width, n.secret = nodes[n.args[0]].width, False
            elif n.op == "load":
                n.width, n.secret = n.imm[0], nodes[n.args[0]].secret
            elif n.op == "layer":
                n.width, n.secret = n.imm[1], True
    for nid in lines:
        n = nodes[nid]
        if n.op in ("add", "sub", "mul"):
            x, y = nodes[n.args[0]], nodes[n.args[1]]
            if x.width != y.width and not ((not x.secret and x.width == 1) or (not y.secret and y.width == 1)):
                raise ProgramError(f"node {nid}: widths {x.width} and {y.width}")
        if n.op in ("lt", "eq") and (nodes[n.args[0]].secret or nodes[n.args[1]].secret):
            raise ProgramError(f"node {nid}: comparison of a secret value")
        if n.op == "bcast" and nodes[n.args[0]].width != 1:
            raise ProgramError(f"node {nid}: bcast of a value of width {nodes[n.args[0]].width}")
        if n.op in ("div", "mod") and nodes[n.args[0]].secret:
            raise ProgramError(f"node {nid}: integer division of a secret value")
        if n.op == "open" and not nodes[n.args[0]].secret:
            raise ProgramError(f"node {nid}: open of a public value")
        if n.op == "load" and (nodes[n.args[1]].secret or nodes[n.args[1]].width != 1):
            raise ProgramError(f"node {nid}: load start must be a public scalar")
        if n.op == "phi" and len({nodes[v].width for v, _ in n.phi}) != 1:
            raise ProgramError(f"node {nid}: phi widths differ")
        if n.op == "layer":
            x, W, b = (nodes[v] for v in n.args)
            din, dout, tr = n.imm
            if (x.width, W.width, b.width) != (din, din * dout, dout) or tr < 1:
                raise ProgramError(f"node {nid}: layer shapes")
            if not (x.secret and W.secret):
                raise ProgramError(f"node {nid}: layer x and W must be secret")
    for b in prog.blocks.values():
        if b.term[0] == "cbr":
            c = nodes[b.term[1]]
            if c.secret or c.width != 1:
                raise ProgramError(f"block {b.id}: branch on a secret or non-scalar condition")


# ---------------------------------------------------------------------------
# sequential execution
# ---------------------------------------------------------------------------
class Exec:
    def __init__(self, prog: Program, p: int, n: int, seed: int, check_seed: int, epoch: int = 0):
        self.prog, self.f, self.n, self.seed = prog, F.Field(p), n, seed
        self.al = self.f.alpha_shares(n, seed)
        self.log = F.MacLog(self.f, n, check_seed, epoch)
        self.val: Dict[int, object] = {}        # node -> Shares (secret) or [L][w] array (public)
        self.count: Dict[int, int] = {}         # executions so far of product / layer nodes
        self.opened: List[np.ndarray] = []
        self.entries = 0

    # public helpers ------------------------------------------------------
    def pub(self, nid: int, width: int) -> np.ndarray:
        v = self.val[nid]
        if v.shape[1] == width:
            return v
        return np.repeat(v, width, axis=1)       # public scalar broadcast

    def share_pub(self, v: np.ndarray) -> F.Shares:
        """Party 0 holds the value, every party alpha_i value as MAC share."""
        f, n = self.f, self.n
        val = np.zeros((n, f.L, v.shape[1]), dtype=np.uint64)
        mac = np.empty_like(val)
        val[0] = v
        for i in range(n):
            mac[i] = f.scale_public(int(F.from_limbs(self.al[i].reshape(f.L, 1))[0]), v)
        return F.Shares(val, mac)

    def add_pub(self, x: F.Shares, v: np.ndarray) -> F.Shares:
        s = self.share_pub(v)
        return self.f.linear(self.al, [x, s], [1, 1])

    def mul_pub(self, x: F.Shares, v: np.ndarray) -> F.Shares:
        f = self.f
        val = np.stack([f.mul_public(x.val[i], v) for i in range(self.n)])
        mac = np.stack([f.mul_public(x.mac[i], v) for i in range(self.n)])
        return F.Shares(val, mac)

    # one node ------------------------------------------------------------
    def run_node(self, nd: Node, pred: Optional[int]):
        f, nodes, p = self.f, self.prog.nodes, self.f.p
        if nd.op == "phi":
            src = [v for v, b in nd.phi if b == pred]
            if not src:
                raise ProgramError(f"phi {nd.id}: no value for predecessor {pred}")
            v = self.at_entry[src[0]]   # the value held when the block was entered
            if nd.secret and not isinstance(v, F.Shares):
                v = self.share_pub(v)
            self.val[nd.id] = v
            return
        if nd.op in ("add", "sub", "mul"):
            a, b = (nodes[i] for i in nd.args)
            va, vb = self.val[a.id], self.val[b.id]
            w = nd.width
            if not nd.secret:
                va, vb = self.pub(a.id, w), self.pub(b.id, w)
                self.val[nd.id] = {"add": f.add_public, "sub": f.sub_public, "mul": f.mul_public}[nd.op](va, vb)
            elif a.secret and b.secret:
                if nd.op == "mul":
                    k = self.count.get(nd.id, 0)
                    self.count[nd.id] = k + 1
                    t = f.deal_triple(self.n, self.seed, triple_array(nd.id, k), w, self.al)
                    z, d, e, dm, em = f.beaver(self.al, va, vb, t)
                    self.log.add(d, dm)
                    self.log.add(e, em)
                    self.opened += [d, e]
                    self.val[nd.id] = z
                else:
                    self.val[nd.id] = f.linear(self.al, [va, vb], [1, 1 if nd.op == "add" else p - 1])
            else:
                sec, pb = (va, self.pub(b.id, w)) if a.secret else (vb, self.pub(a.id, w))
                if nd.op == "mul":
                    self.val[nd.id] = self.mul_pub(sec, pb)
                elif nd.op == "add":
                    self.val[nd.id] = self.add_pub(sec, pb)
                elif a.secret:   # secret - public
                    self.val[nd.id] = self.add_pub(sec, f.sub_public(np.zeros_like(pb), pb))
                else:            # public - secret
                    self.val[nd.id] = self.add_pub(f.linear(self.al, [sec], [p - 1]), pb)
        elif nd.op in ("lt", "eq"):
            w = nd.width
            xa = F.from_limbs(self.pub(nd.args[0], w))
            xb = F.from_limbs(self.pub(nd.args[1], w))
            r = [int(u < v) if nd.op == "lt" else int(u == v) for u, v in zip(xa, xb)]
            self.val[nd.id] = F.to_limbs(r, f.L)
        elif nd.op == "cat":   # the lanes of the first value, then those of the second
            parts = [self.val[i] for i in nd.args]
            if nd.secret:
                parts = [v if isinstance(v, F.Shares) else self.share_pub(v) for v in parts]
                self.val[nd.id] = F.Shares(np.concatenate([v.val for v in parts], axis=2),
                                           np.concatenate([v.mac for v in parts], axis=2))
            else:
                self.val[nd.id] = np.concatenate(parts, axis=1)
        elif nd.op == "bcast":
            v, w = self.val[nd.args[0]], nd.imm[0]
            if nd.secret:
                self.val[nd.id] = F.Shares(np.repeat(v.val, w, axis=2), np.repeat(v.mac, w, axis=2))
            else:
                self.val[nd.id] = np.repeat(v, w, axis=1)
        elif nd.op in ("div", "mod"):   # a public value as an integer in [0, p) by a literal
            k = nd.imm[0]
            xa = F.from_limbs(self.val[nd.args[0]])
            self.val[nd.id] = F.to_limbs([int(u) // k if nd.op == "div" else int(u) % k for u in xa], f.L)
        elif nd.op == "reduce":
            v = self.val[nd.args[0]]
            if nd.secret:
                self.val[nd.id] = f.reduce_add(v)
            else:
                s = 0
                for u in F.from_limbs(v):
                    s = (s + u) % p
                self.val[nd.id] = F.to_limbs([s], f.L)
        elif nd.op == "open":
            x = self.val[nd.args[0]]
            o = f.open(x.val)
            self.log.add(o, x.mac)
            self.opened.append(o)
            self.val[nd.id] = o
        elif nd.op == "load":
            base = self.val[nd.args[0]]
            s = F.from_limbs(self.val[nd.args[1]])[0]
            cnt = nd.imm[0]
            bw = nodes[nd.args[0]].width
            if s + cnt > bw:
                raise ProgramError(f"load {nd.id}: elements {s}..{s + cnt - 1} beyond width {bw}")
            if isinstance(base, F.Shares):
                self.val[nd.id] = F.Shares(np.ascontiguousarray(base.val[:, :, s:s + cnt]),
                                           np.ascontiguousarray(base.mac[:, :, s:s + cnt]))
            else:
                self.val[nd.id] = np.ascontiguousarray(base[:, s:s + cnt])
        elif nd.op == "layer":
            from .pipelines import DealtLayer, deal_matvec_triple, linear_layer_tile
            din, dout, tr = nd.imm
            k = self.count.get(nd.id, 0)
            self.count[nd.id] = k + 1
            T = deal_matvec_triple(f, self.n, self.seed, triple_array(nd.id, k), dout, din, tr, self.al)
            x, W, b = (self.val[i] for i in nd.args)
            if not nodes[nd.args[2]].secret:   # a public bias is a public constant of the sum
                b = self.share_pub(self.pub(nd.args[2], dout))
            D = DealtLayer(f, self.n, self.seed, dout, din, tr, self.al, None, W, None, x, None, b, T)
            yv, ym = [], []
            for t in range(D.n_tiles):
                Dt, Et, yt = linear_layer_tile(D, t, self.log)
                self.opened += [Dt, Et]
                yv.append(yt.val)
                ym.append(yt.mac)
            self.val[nd.id] = F.Shares(np.concatenate(yv, axis=2), np.concatenate(ym, axis=2))
        else:
            raise ProgramError(f"cannot execute {nd.op}")

    def run(self):
        prog, f = self.prog, self.f
        for nid, nd in prog.nodes.items():
            if nd.op == "input":
                if nd.secret:
                    self.val[nid] = f.deal_uniform_secret(self.n, self.seed, nd.imm[0], nd.width, self.al)[1]
                else:
                    self.val[nid] = f.deal_values(self.seed, nd.imm[0], nd.width)
            elif nd.op == "const":
                self.val[nid] = F.to_limbs(nd.imm * nd.width if len(nd.imm) == 1 else list(nd.imm), f.L)
        blk, pred = prog.entry, None
        while True:
            self.entries += 1
            if self.entries > MAX_BLOCK_ENTRIES:
                raise ProgramError("too many block entries")
            b = prog.blocks[blk]
            self.at_entry = dict(self.val)   # phis read these, all at once
            for nid in b.lines:
                self.run_node(prog.nodes[nid], pred)
            if b.term[0] == "ret":
                break
            if b.term[0] == "br":
                nxt = b.term[1]
            else:
                c = F.from_limbs(self.val[b.term[1]])[0]
                nxt = b.term[2] if c != 0 else b.term[3]
            pred, blk = blk, nxt
        ok, sigma = self.log.check(self.al)
        return dict(outputs={o: self.val[o] for o in prog.outputs}, ok=ok, sigma=sigma,
                    opened=self.opened, entries=self.entries, alpha=self.al)


def run_program(text: str, p: int, n: int, seed: int, check_seed: int, epoch: int = 0):
    return Exec(parse(text, p), p, n, seed, check_seed, epoch).run()
