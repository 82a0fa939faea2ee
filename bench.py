"""Benchmark of the SPDZ online-phase hot path on one MI355X.

One step = the fused pipeline on 3 simulated parties over p = 2^127 - 1 with
2^24-element secret vectors: Beaver product z = x*y (mask, open d and e,
recombine), w = z + 3x - y, open(w), s = ReduceAdd(z) (the secret dot product
sum x_i y_i), open(s), and the MAC check over every opened value with its
verdict read back on the host.  Inputs (shares, MAC shares, triples) are dealt
on the device before the timed region and stay resident in HBM.

Prints one JSON line.  `value` is MAC'd Beaver multiplications per second
(elements of the batch per second of whole-step wall time).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per element of the fused pipeline kernel: reads x, y, a, b, c
# (values and MAC shares, 10 n L words), writes z and w (4 n L words) and the
# public d, e, w (3 L words): (14 n + 3) * 8 L bytes
def fused_bytes_per_elem(n: int, L: int) -> int:
    return (14 * n + 3) * 8 * L


def beaver_bytes_per_elem(n: int, L: int) -> int:
    return 12 * n * 8 * L   # reads 10 n L words, writes z (2 n L words)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "beaver_fused_n3_p127_w16777216_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2512_11112_amd", "csrc", f) for f in ("elementwise.hip", "field.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(W: int):
    """HBM bytes per launch from the committed counter summary, if it was taken on the current kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m_hash = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    m_w = re.search(r"width:\s*(\d+)", txt)
    if not (m_hash and m_bytes and m_w) or m_hash.group(1) != kernel_source_hash() or int(m_w.group(1)) != W:
        return None
    return float(m_bytes.group(1))


def cpu_baseline(p: int, n: int, W_sample: int, seed: int):
    """The oracle (tier-1 C, OpenMP over all host threads) on a bounded sample of the same pipeline."""
    from oracle.pipelines import deal_elementwise, pipeline_run
    D = deal_elementwise(p, n, W_sample, seed)
    t0 = time.perf_counter()
    r = pipeline_run(D, check_seed=seed)
    dt = time.perf_counter() - t0
    assert r["ok"]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": W_sample / dt, "unit": "mults/s", "cores": threads, "kind": "oracle",
            "sample": f"{W_sample} of {1 << 24} elements, whole pipeline (Beaver, linear, ReduceAdd, "
                      f"opens, MAC check) on the oracle (plain C, generic long-division mod p), "
                      f"{dt:.2f} s wall, dealing excluded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--width", type=int, default=1 << 24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 22)
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the build simulates all parties on one device "
              f"(--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_11112_amd import spdz as S
    from workloads import ARR_A, ARR_X, ARR_Y, P61, P127, SEEDS_TIMING

    p, n, W, seed = P127, 3, args.width, SEEDS_TIMING[0]
    L = S.n_limbs(p)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    alpha = S.deal_alpha(p, n, seed)
    ctx = S.Context(n, p, alpha, check_seed=seed, stream=stream)
    x, y, z, w = (ctx.new_shares(W) for _ in range(4))
    s = ctx.new_shares(1)
    t = S.TripleTensor.empty(n, L, W)
    ctx.spdz_deal_secret(seed, ARR_X, x)
    ctx.spdz_deal_secret(seed, ARR_Y, y)
    ctx.spdz_deal_triple(seed, ARR_A, t)
    d_pub, e_pub, w_pub = ctx.new_public(W), ctx.new_public(W), ctx.new_public(W)
    lin = (1, 3, p - 1, 0)

    def step():
        ctx.spdz_mul_fused(x, y, t, z, d_pub, e_pub, lin=lin, w=w, w_pub=w_pub, s=s)
        ctx.spdz_open(s)
        ok, _ = ctx.spdz_mac_check()
        if not ok:
            raise RuntimeError("MAC check rejected an honest run")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.spdz_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    k_ms, k_cnt = ctx.spdz_timing_get("beaver_fused")
    ctx.spdz_timing_enable(False)
    k_avg_ms = k_ms / max(k_cnt, 1)
    alg_bytes = fused_bytes_per_elem(n, L) * W
    achieved = alg_bytes / (k_avg_ms * 1e-3) / 1e9
    traffic = read_traffic(W)

    out = {
        "metric": "MAC'd Beaver mults/s mod p at 1 GPU + % HBM peak",
        "value": W / (ms_step * 1e-3),
        "unit": "mults/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"beaver_linear_dot_n3_p127_w{W}", "parties": n, "modulus": "2^127-1",
                   "limbs": L, "width": W, "pipeline": "z=x*y; w=z+3x-y; open(w); s=sum(z); open(s); mac_check",
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "kernel": "k_beaver<F127,3,fused>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel_ms": k_avg_ms, "launches": k_cnt,
                     "alg_bytes_per_launch": alg_bytes},
    }
    del x, y, z, w, t, d_pub, e_pub, w_pub
    ctx.close()
    torch.cuda.empty_cache()

    if not args.no_extras:
        out["extra"] = extras(torch, S)
        out["roofline"]["frac_of_copy"] = achieved / out["extra"]["copy_GBps"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, n, args.cpu_sample, seed)
    print(json.dumps(out), flush=True)


def extras(torch, S):
    """Plain-copy bandwidth, the plain Beaver kernel at 2 parties over 2^61-1, and the
    2^16-element configuration's step latency."""
    from workloads import ARR_A, ARR_X, ARR_Y, P61, SEEDS_TIMING
    res = {}
    words = 1 << 28
    a = torch.empty(words, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        S.spdz_copy_probe(b, a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        S.spdz_copy_probe(b, a)
    e1.record()
    torch.cuda.synchronize()
    res["copy_GBps"] = 2 * words * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    for W in (1 << 24, 1 << 16):
        p, n, seed = P61, 2, SEEDS_TIMING[0]
        ctx = S.Context(n, p, S.deal_alpha(p, n, seed), check_seed=seed)
        x, y, z = (ctx.new_shares(W) for _ in range(3))
        t = S.TripleTensor.empty(n, 1, W)
        ctx.spdz_deal_secret(seed, ARR_X, x)
        ctx.spdz_deal_secret(seed, ARR_Y, y)
        ctx.spdz_deal_triple(seed, ARR_A, t)

        def step():
            ctx.spdz_mul_batch(x, y, t, z)
            ok, _ = ctx.spdz_mac_check()
            assert ok
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        ctx.spdz_timing_enable(True)
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        kms, kc = ctx.spdz_timing_get("beaver")
        kavg = kms / max(kc, 1)
        tag = "p61_n2_w2^24" if W == 1 << 24 else "p61_n2_w2^16"
        res[f"beaver_{tag}_step_ms"] = ms
        res[f"beaver_{tag}_mults_per_s"] = W / (ms * 1e-3)
        res[f"beaver_{tag}_kernel_ms"] = kavg
        res[f"beaver_{tag}_kernel_GBps"] = beaver_bytes_per_elem(n, 1) * W / (kavg * 1e-3) / 1e9
        ctx.close()
        del x, y, z, t
        torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
