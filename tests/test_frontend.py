"""The LLVM front end (paper_2512_11112_amd/frontend.py) on the CPU.

Each test program under tests/frontend/ is compiled twice:
  * by the front end: clang -O2 (with the paper's vectorizer flags where given), the IR read
    into the runtime's program text, which the oracle's interpreter runs on shares;
  * as C++ with word_t an element of F_p (tests/frontend/clear.hpp), an independent cleartext
    evaluation of the same C function on the same input values.
The opened result of the program must equal the cleartext function's return value.  The IR
structure the paper describes is checked on the way: privacy read from the annotations, Load
views with their lane counts, one layer node for mark_linear_layer, blocks and branches.
"""
import ctypes
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle.fast as F
from oracle.program import run_program
from paper_2512_11112_amd import frontend as FE
from workloads import P_PAPER

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "frontend")

pytestmark = pytest.mark.skipif(not os.path.exists(FE.CLANG), reason="clang not installed")


def source(name):
    with open(os.path.join(HERE, name)) as fh:
        return fh.read()


def cleartext_function(name, func, defines=None):
    """The C function compiled as C++ over F_p (clear.hpp), loaded with ctypes."""
    d = tempfile.mkdtemp()
    wrap = os.path.join(d, "wrap.cpp")
    with open(wrap, "w") as fh:
        fh.write(f'extern "C" {{\n#include "{os.path.join(HERE, name)}"\n}}\n')
    so = os.path.join(d, "clear.so")
    cxx = shutil.which("g++") or shutil.which("clang++")
    cmd = [cxx, "-O1", "-shared", "-fPIC", "-std=c++17", "-include", os.path.join(HERE, "clear.hpp"), wrap, "-o", so]
    cmd += [f"-D{k}={v}" for k, v in (defines or {}).items()]
    subprocess.run(cmd, check=True, capture_output=True)
    return getattr(ctypes.CDLL(so), func)


def input_values(t, sizes, seed, p=P_PAPER):
    """Values the oracle deals for each input of the program (parameter k is array k)."""
    f = F.Field(p)
    out = {}
    for k, nid in t.inputs.items():
        m = re.search(rf"^input {nid} (private|public) (\d+) {k}$", t.text, flags=re.M)
        out[k] = [int(v) for v in F.from_limbs(f.deal_values(seed, k, int(m.group(2))))]
    return out


def opened(t, res):
    return [int(v) for v in F.from_limbs(res["outputs"][t.revealed])]


def u64_array(vals):
    return (ctypes.c_uint64 * len(vals))(*vals)


@pytest.mark.parametrize("din,dout", [(8, 4), (37, 11)])
def test_fig2_linear_layer(din, dout):
    defines = {"DIN": din, "DOUT": dout}
    t = FE.translate(source("fig2_layer.c"), "linear_layer", sizes={0: din, 1: din * dout, 2: dout},
                     defines=defines)
    assert t.privacy == {0: "private", 1: "private", 2: "public"}
    layers = re.findall(r"^(\d+) = layer (\d+) (\d+) (\d+) (\d+) (\d+) (\d+)$", t.text, flags=re.M)
    assert len(layers) == 1 and layers[0][4:6] == (str(din), str(dout))
    seed = 3
    res = run_program(t.text, P_PAPER, 2, seed, seed)
    assert res["ok"]
    vals = input_values(t, {}, seed)
    fn = cleartext_function("fig2_layer.c", "linear_layer", defines)
    fn.restype = ctypes.POINTER(ctypes.c_uint64)
    fn.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 3
    y = fn(u64_array(vals[0]), u64_array(vals[1]), u64_array(vals[2]))
    assert opened(t, res) == [y[r] for r in range(dout)]
    # and W x + b written out in Python integers
    x, W, b = vals[0], vals[1], vals[2]
    assert opened(t, res) == [(sum(W[r * din + k] * x[k] for k in range(din)) + b[r]) % P_PAPER for r in range(dout)]


@pytest.mark.parametrize("n,width,vw,il", [(37, 40, None, None), (64, 64, 16, 2), (100, 128, 4, 4), (3, 8, None, None)])
def test_public_bound_loop(n, width, vw, il):
    """The loop bound is a public parameter bound at translation time; vectorized loads are
    Load views of vw lanes and the remainder loop runs element by element."""
    t = FE.translate(source("dot_loop.c"), "dot", sizes={0: width, 1: width}, bind={2: n}, vector_width=vw,
                     interleave=il)
    assert t.privacy == {0: "private", 1: "private", 2: "public"}
    counts = {int(c) for c in re.findall(r"= load \d+ \d+ (\d+)$", t.text, flags=re.M)}
    if vw and n >= vw * (il or 1):
        assert vw in counts
    assert "cbr" in t.text          # the loop's back edge is a public branch
    seed = 8
    res = run_program(t.text, P_PAPER, 2, seed, seed)
    assert res["ok"]
    vals = input_values(t, {}, seed)
    fn = cleartext_function("dot_loop.c", "dot")
    fn.restype = ctypes.c_uint64
    fn.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 2 + [ctypes.c_uint32]
    want = fn(u64_array(vals[0]), u64_array(vals[1]), n)
    assert opened(t, res) == [want]
    x, y = vals[0], vals[1]
    assert want == sum(x[i] * y[i] + 3 * x[i] for i in range(n)) % P_PAPER


@pytest.mark.parametrize("vw,il", [(16, 2), (4, 4), (None, None)])
@pytest.mark.parametrize("seed", [8, 11])
def test_runtime_bound_loop(vw, il, seed):
    """The bound is a public input known only at run time: the vectorizer's trip-count
    arithmetic (the bound rounded down to a multiple of the vector length, an and with a mask)
    becomes the program's public div/mod, and the remainder loop takes what is left."""
    t = FE.translate(source("dot_runtime.c"), "dot_rt", sizes={0: 4096, 1: 4096}, vector_width=vw, interleave=il)
    assert t.privacy == {0: "private", 1: "private", 2: "public"} and 2 in t.inputs
    assert re.search(r"= mod \d+ \d+$", t.text, flags=re.M)
    res = run_program(t.text, P_PAPER, 2, seed, seed)
    assert res["ok"]
    vals = input_values(t, {}, seed)
    n = vals[2][0]
    fn = cleartext_function("dot_runtime.c", "dot_rt")
    fn.restype = ctypes.c_uint64
    fn.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 2 + [ctypes.c_uint32]
    want = fn(u64_array(vals[0]), u64_array(vals[1]), n)
    assert opened(t, res) == [want]
    x, y = vals[0], vals[1]
    assert want == sum(x[i] * y[i] + 3 * x[i] for i in range(n % 4001)) % P_PAPER


@pytest.mark.parametrize("din,dout,vw", [(64, 32, 16), (64, 32, None), (100, 7, None), (128, 16, 8)])
def test_nested_loops_over_rows(din, dout, vw):
    """Rows addressed by a variable byte offset into the matrix, the inner dot product unrolled
    and vectorized (blocks lowered in dominance order: at -O2 a value's definition can follow its
    use in the text): sum_r (W_r . x)^2 equals the cleartext build and Python integers."""
    defines = {"DIN": din, "DOUT": dout}
    t = FE.translate(source("matvec.c"), "matvec_sum", sizes={0: din * dout, 1: din}, defines=defines,
                     vector_width=vw)
    assert "cbr" in t.text or dout == 1
    seed = 13
    res = run_program(t.text, P_PAPER, 2, seed, seed)
    assert res["ok"]
    vals = input_values(t, {}, seed)
    fn = cleartext_function("matvec.c", "matvec_sum", defines)
    fn.restype = ctypes.c_uint64
    fn.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 2
    want = fn(u64_array(vals[0]), u64_array(vals[1]))
    assert opened(t, res) == [want]
    W, x = vals[0], vals[1]
    assert want == sum(sum(W[r * din + k] * x[k] for k in range(din)) ** 2 for r in range(dout)) % P_PAPER


@pytest.mark.parametrize("vw", [8, None])
def test_secret_scalar_broadcast(vw):
    """A secret scalar parameter multiplied into vectors becomes the program's bcast."""
    t = FE.translate(source("axpy.c"), "axpy_dot", sizes={0: 64, 1: 64}, vector_width=vw)
    assert re.search(r"= bcast \d+ \d+$", t.text, flags=re.M)
    seed = 17
    res = run_program(t.text, P_PAPER, 2, seed, seed)
    assert res["ok"]
    vals = input_values(t, {}, seed)
    fn = cleartext_function("axpy.c", "axpy_dot")
    fn.restype = ctypes.c_uint64
    fn.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 2 + [ctypes.c_uint64]
    want = fn(u64_array(vals[0]), u64_array(vals[1]), vals[2][0])
    assert opened(t, res) == [want]
    x, y, a = vals[0], vals[1], vals[2][0]
    assert want == sum((a * x[i] + y[i]) ** 2 for i in range(64)) % P_PAPER


@pytest.mark.parametrize("tval", [2, 9])
def test_public_branch(tval):
    """Both sides are loops, so the branch stays a conditional br on a public comparison, the
    sides join in a phi; the tail multiplies by 2^3 (a shl) and subtracts a constant."""
    t = FE.translate(source("branch.c"), "branchy", sizes={0: 64, 1: 64}, bind={2: tval}, vector_width=8)
    # with the bound parameter the comparison folds away: one side is never entered
    seed = 4
    res = run_program(t.text, P_PAPER, 3, seed, seed)
    assert res["ok"]
    vals = input_values(t, {}, seed)
    fn = cleartext_function("branch.c", "branchy")
    fn.restype = ctypes.c_uint64
    fn.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 2 + [ctypes.c_uint32]
    assert opened(t, res) == [fn(u64_array(vals[0]), u64_array(vals[1]), tval)]
    # unbound, the condition is a public input compared at run time: a real two-way branch
    t2 = FE.translate(source("branch.c"), "branchy", sizes={0: 64, 1: 64}, vector_width=8)
    assert re.search(r"= lt ", t2.text) and re.search(r"^cbr ", t2.text, flags=re.M)
    assert "phi" in t2.text
    res2 = run_program(t2.text, P_PAPER, 2, seed, seed)
    tv = input_values(t2, {}, seed)[2][0]
    assert opened(t2, res2) == [fn(u64_array(vals[0]), u64_array(vals[1]), tv % (1 << 32))]


@pytest.mark.parametrize("c", [1, 7])
def test_scalars_select_and_shift(c):
    t = FE.translate(source("poly.c"), "poly", sizes={0: 4}, bind={2: c})
    assert t.privacy == {0: "private", 1: "private", 2: "public"}
    seed = 6
    res = run_program(t.text, P_PAPER, 2, seed, seed)
    vals = input_values(t, {}, seed)
    fn = cleartext_function("poly.c", "poly")
    fn.restype = ctypes.c_uint64
    fn.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64, ctypes.c_uint32]
    assert opened(t, res) == [fn(u64_array(vals[0]), vals[1][0], c)]
    # with c unbound the select stays in the program, on a public condition
    t2 = FE.translate(source("poly.c"), "poly", sizes={0: 4})
    assert re.search(r"= select ", t2.text) or re.search(r"^cbr ", t2.text, flags=re.M)
    res2 = run_program(t2.text, P_PAPER, 2, seed, seed)
    cv = input_values(t2, {}, seed)[2][0]
    assert opened(t2, res2) == [fn(u64_array(vals[0]), vals[1][0], cv % (1 << 32))]


def test_privacy_taint_reaches_loop_carried_values():
    """The accumulator phi of the vectorized loop depends on private inputs only through its
    back edge: the fixed point marks it secret and the returned value is opened."""
    ll = FE.compile_ir(source("dot_loop.c"), vector_width=4)
    f = FE.parse_ir(ll)["dot"]
    sec = FE.taint(f, {0: "private", 1: "private", 2: "public"})
    phis = [s.split("=")[0].strip() for _, ins in f.blocks for s in ins if "= phi <4 x i32>" in s]
    assert phis and all(ph in sec for ph in phis)
    idx = [s.split("=")[0].strip() for _, ins in f.blocks for s in ins if "= phi i64" in s]
    assert idx and not any(ix in sec for ix in idx)


def test_rejections():
    src = source("rejected.c")
    with pytest.raises(FE.FrontendError, match="secret"):
        FE.translate(src, "secret_branch", sizes={0: 8})
    with pytest.raises(FE.FrontendError, match="store"):
        FE.translate(src, "stores", sizes={0: 16})
    with pytest.raises(FE.FrontendError, match="annotation"):
        FE.translate("word_t f(const word_t *x) { return x[0] * x[1]; }", "f", sizes={0: 2})
    # integer operations exist only for public values: bits of a secret have no arithmetic form
    with pytest.raises(FE.FrontendError, match="secret"):
        FE.translate(src, "secret_shift", sizes={0: 2})
    with pytest.raises(FE.FrontendError, match="secret"):
        FE.translate(src, "secret_mask", sizes={0: 2})
    # a public and with a mask that is not one run of one bits
    with pytest.raises(FE.FrontendError, match="mask"):
        FE.translate(src, "public_odd_mask", sizes={0: 128})


def test_ir_reader_on_the_papers_listing_shape():
    """Vector loads through a GEP chain with byte offsets (the IR shape of Fig. 3) become Load
    views whose start adds the element offset."""
    ll = """
define dso_local i32 @g(ptr noundef %0, i64 noundef %1) local_unnamed_addr #0 {
  %3 = alloca ptr, align 8
  %4 = alloca i64, align 8
  %5 = getelementptr inbounds i32, ptr %0, i64 %1
  %6 = load <128 x i32>, ptr %5, align 4, !tbaa !6
  %7 = getelementptr inbounds i8, ptr %5, i64 512
  %8 = load <128 x i32>, ptr %7, align 4, !tbaa !6
  %9 = add <128 x i32> %6, %8
  %10 = tail call i32 @llvm.vector.reduce.add.v128i32(<128 x i32> %9)
  ret i32 %10
}
"""
    f = FE.parse_ir(ll)["g"]
    low = FE._Lower(f, {0: "private", 1: "public"}, {0: 1024}, {1: 256}, P_PAPER, 524280)
    text, _, revealed = low.run()
    loads = re.findall(r"^(\d+) = load (\d+) (\d+) 128$", text, flags=re.M)
    assert len(loads) == 2
    consts = dict((int(i), int(v)) for i, v in re.findall(r"^const (\d+) 1 (\d+)$", text, flags=re.M))
    starts = []
    for _, _, s in loads:
        s = int(s)
        if s in consts:
            starts.append(consts[s])
        else:   # start + offset
            m = re.search(rf"^{s} = add (\d+) (\d+)$", text, flags=re.M)
            starts.append(consts[int(m.group(1))] + consts[int(m.group(2))])
    assert sorted(starts) == [256, 384]
    assert re.search(r"= reduce ", text) and revealed is not None


RANDOM_C_SEEDS = range(60)


@pytest.fixture(scope="module")
def random_c_outcomes():
    """Each seeded random C function (tests/frontend/random_c.py) translated and run by the
    oracle's interpreter next to its cleartext build: 'ok', or the front end's refusal."""
    import sys
    sys.path.insert(0, HERE)
    from random_c import random_c
    out = {}
    d = tempfile.mkdtemp()
    for seed in RANDOM_C_SEEDS:
        src = random_c(seed)
        try:
            t = FE.translate(src, "fz", sizes={0: 64, 1: 64}, vector_width=[None, 4, 8][seed % 3])
        except FE.FrontendError as e:
            out[seed] = f"refused: {e}"
            continue
        res = run_program(t.text, P_PAPER, 2, seed, seed)
        vals = input_values(t, {}, seed)
        path = os.path.join(d, f"fz{seed}.c")
        with open(path, "w") as fh:
            fh.write(src)
        fn = cleartext_function(path, "fz")
        fn.restype = ctypes.c_uint64
        fn.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 2 + [ctypes.c_uint64, ctypes.c_uint32]
        tv = vals[3][0] if 3 in vals else 0
        want = fn(u64_array(vals[0]), u64_array(vals[1]), vals[2][0], tv % (1 << 32))
        out[seed] = "ok" if res["ok"] and opened(t, res) == [want] else f"wrong: {opened(t, res)} != {want}"
    return out


def test_random_c_functions(random_c_outcomes):
    """Random straight-line code, vectorized dot-product loops, Horner loops, public branches,
    selects of values and of pointers, and loops bounded by a mask of a public parameter: every
    function the front end accepts computes the cleartext result; the rest are refused by name
    (no translation runs and gives a wrong value)."""
    wrong = {s: o for s, o in random_c_outcomes.items() if o.startswith("wrong")}
    assert not wrong, wrong
    ok = sum(o == "ok" for o in random_c_outcomes.values())
    print(f"{ok} of {len(random_c_outcomes)} accepted", flush=True)
    assert ok >= 3 * len(random_c_outcomes) // 4
