#!/usr/bin/env python3
"""Benchmark: secure int64-ring GEMM on one MI355X.

One step is one pass of the whole hot path over one 4096x4096x4096 problem
with inputs resident in HBM: both operands secret-shared (PRZS), a fresh
matrix Beaver triple from the dealer, the Beaver matmul (mask, device-local
open, each party's finish GEMM with fused 2^16 truncation) in the limb (INT8
matrix core) form, and the reveal.  `value` is plaintext-equivalent ring
operations 2*M*N*K per step divided by the step time (Tops/s).

Also reported (outside the timed region): the ring GEMM alone in both forms
and the limb form's speedup, the Beaver element-wise product rate against
HBM bandwidth, the secure MLP (784-1024-1024-10, batch 128) latency, the
roofline of the dominant kernel from HIP events around every GEMM launch,
and the CPU oracle timed on a bounded slice of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("secure int64-ring GEMM Tops/s (limb-MFMA vs plain, bit-exact); Beaver mul elem/s")
INT8_PEAK_TOPS = 5000.0  # MI355X dense INT8 matrix peak, 5.0 POP/s
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
M = N = K = 4096
FRAC = 16


def log(*a):
    print(*a, file=sys.stderr, flush=True)


EXTRAS = ("ceilings", "small", "ring_gemm", "beaver_mul", "mlp", "sweep", "multiparty", "binary", "grouped", "grouped_mul",
          "conv", "power")
# run only when named: for profiling runs
OPT_EXTRAS = ("grouped_schedules",)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="limb8", choices=["limb8", "plain"])
    ap.add_argument("--triples", default="packed", choices=["packed", "plain"],
                    help="limb form: the dealer also packs the triple's a1, b0, b1 (offline), so that the online "
                         "Beaver matmul packs only eps, a0 + eps and delta; or a plain triple")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--extra", action="append", choices=EXTRAS + OPT_EXTRAS, metavar="NAME",
                    help="run only these secondary measurements (repeatable): " + ", ".join(EXTRAS) +
                         "; only when named: " + ", ".join(OPT_EXTRAS))
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="after the JSON line, run three device-to-device copies of MIB MiB "
                         "(a plain copy kernel of known size, to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU, which holds both parties' shares; --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        return 2

    import torch
    import paper_2109_00984_amd as mpc
    import workloads

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    data_seed, party_seed, dealer_seed = workloads.seeds(3)
    ctx = mpc.Context(device=0, seed=party_seed)
    dev = torch.device("cuda", 0)

    def to_dev(a):
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(dev)

    log("bench: generating 4096x4096 uniform uint64 operands")
    Xh = workloads.uniform_u64(data_seed, (M, K))
    Yh = workloads.uniform_u64(data_seed + 1, (K, N))
    X, Y = to_dev(Xh), to_dev(Yh)
    x = mpc.SharedPair(ctx.empty((M, K)), ctx.empty((M, K)))
    y = mpc.SharedPair(ctx.empty((K, N)), ctx.empty((K, N)))
    t = mpc.TripleShares(ctx.empty((M, K)), ctx.empty((M, K)), ctx.empty((K, N)),
                         ctx.empty((K, N)), ctx.empty((M, N)), ctx.empty((M, N)))
    z = mpc.SharedPair(ctx.empty((M, N)), ctx.empty((M, N)))
    r = ctx.empty((M, N))
    dims = (M, N, K)
    packed_triples = args.form == "limb8" and args.triples == "packed"
    packed = torch.empty(ctx.packed_triple_bytes(M, N, K), dtype=torch.uint8, device=dev) if packed_triples else None

    def step():
        ctx.share(X, 0, 1, out=x)
        ctx.share(Y, 1, 2, out=y)
        if packed_triples:
            ctx._dealer_packed_into(dealer_seed, 3, dims, t, packed)
            ctx.beaver_matmul_prepacked(x, y, t, packed, FRAC, out=z)
        else:
            ctx.dealer_into(mpc.TRIPLE_MATMUL, dealer_seed, 3, dims, t)
            ctx.beaver_matmul(x, y, t, FRAC, args.form, out=z)
        ctx.reveal(z, out=r)

    ctx.profile(True)
    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    ctx.sync()
    ctx.profile_read()  # clear
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    elapsed = t1 - t0
    ms_per_step = elapsed / args.steps * 1e3
    value = 2.0 * M * N * K * args.steps / elapsed / 1e12
    log(f"bench: {ms_per_step:.3f} ms/step, {value:.2f} Tops/s")

    # dominant kernel: the ring GEMM launches of the timed region
    g = prof[args.form]
    avg_ms = g["total_ms"] / max(1, g["launches"])
    if args.form == "limb8":
        per_launch_ops = 72.0 * g["ring_macs"] / max(1, g["launches"])  # 36 int8 MACs per ring MAC
        achieved = per_launch_ops / (avg_ms * 1e-3) / 1e12
        tile = ctx.default_tile_config()
        kernel = "k_limb_gemm_lds" if tile["variant"].startswith("lds") else "k_limb_gemm"
        traffic, alg_bytes = measured_traffic(kernel)
        roofline = {"bound": "mfma", "achieved": round(achieved, 1), "peak": INT8_PEAK_TOPS,
                    "unit": "TOP/s", "frac": round(achieved / INT8_PEAK_TOPS, 4),
                    "traffic": traffic, "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE "
                    "+ WRITE_SIZE, copy-calibrated)", "algorithmic_bytes_per_launch": alg_bytes,
                    "kernel": kernel, "tile": tile["variant"], "launches": g["launches"],
                    "avg_launch_ms": round(avg_ms, 4),
                    "work_per_launch": "72 int8 ops per ring multiply-accumulate (36 limb pairs)"}
    else:
        per_launch_ops = 2.0 * g["ring_macs"] / max(1, g["launches"])
        achieved = per_launch_ops / (avg_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": None,
                    "unit": "Tops/s (ring)", "frac": None, "traffic": None,
                    "kernel": "k_plain_gemm", "launches": g["launches"],
                    "avg_launch_ms": round(avg_ms, 4)}

    # the final step's output, for the CPU-oracle leg to compare against
    z_rows = (z.s0.cpu().numpy().view(np.uint64), z.s1.cpu().numpy().view(np.uint64))

    extras = {}
    if not args.no_extras:
        extras = secondary(ctx, mpc, torch, workloads, X, Y, set(args.extra or EXTRAS), cpu=not args.no_cpu)
        if "ceiling_mfma_i8_random_TOPs" in extras and args.form == "limb8":
            # the dominant kernel against the sustained matrix-core rate on random data
            extras["gemm_frac_of_mfma_random_ceiling"] = round(
                roofline["achieved"] / extras["ceiling_mfma_i8_random_TOPs"], 4)
        if "ceiling_hbm_stream_10r2w_GBps" in extras and "beaver_mul_hbm_GBps_algorithmic" in extras:
            # the fused Beaver product against its own access pattern with trivial arithmetic
            extras["beaver_mul_frac_of_stream_ceiling"] = round(
                extras["beaver_mul_hbm_GBps_algorithmic"] / extras["ceiling_hbm_stream_10r2w_GBps"], 4)
        if "ceiling_hbm_stream_10r2w_2e28_GBps" in extras and "beaver_mul_sweep" in extras:
            # the largest sweep point against the same pattern at the same size
            extras["beaver_mul_2e28_frac_of_stream_ceiling"] = round(
                extras["beaver_mul_sweep"]["2^28"]["GBps"] / extras["ceiling_hbm_stream_10r2w_2e28_GBps"], 4)
        if "ceiling_valu_ring_TMACs" in extras and "ring_gemm_4096_plain_ms" in extras:
            extras["plain_gemm_frac_of_valu_ceiling"] = round(
                M * N * K / (extras["ring_gemm_4096_plain_ms"] * 1e-3) / 1e12 / extras["ceiling_valu_ring_TMACs"], 4)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(Xh, Yh, party_seed, dealer_seed, z_rows)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Tops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic (uniform uint64 operands, seeded)",
        "config": {"workload": "secure ring GEMM 4096x4096x4096 over Z/2^64: share both "
                               "operands, dealer matrix triple, Beaver matmul with 2^16 "
                               "truncation, reveal",
                   "M": M, "N": N, "K": K, "form": args.form, "frac_bits": FRAC,
                   "triples": "offline-packed" if packed_triples else "plain",
                   "parties": 2, "parallelism": "single GPU, two party streams"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    if args.copy_calibrate > 0:
        n = args.copy_calibrate << 17  # int64 elements
        src = torch.empty(n, dtype=torch.int64, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration, 3 x {args.copy_calibrate} MiB device-to-device")
    ctx.close()
    return 0


def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", f"{kernel}_secure_gemm_4096_traffic.md")


LIMB_SOURCE = os.path.join(ROOT, "paper_2109_00984_amd", "csrc", "gemm_limb.hip")
API_SOURCE = os.path.join(ROOT, "paper_2109_00984_amd", "csrc", "api.cpp")


def kernel_fingerprint():
    """sha256 over the limb GEMM source (comments and blank space dropped) and
    the library's default tile schedule: the two things the GEMM's HBM traffic
    depends on."""
    import hashlib
    import re
    src = open(LIMB_SOURCE).read()
    src = re.sub(r"//[^\n]*", "", src)
    src = "\n".join(" ".join(ln.split()) for ln in src.splitlines() if ln.strip())
    h = hashlib.sha256(src.encode())
    sched = [ln.strip() for ln in open(API_SOURCE).read().splitlines() if "TileSched sched_default" in ln]
    h.update("\n".join(sched).encode())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per limb-GEMM launch of this workload (and the algorithmic
    bytes beside them), from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, each counter scaled by its reading on a copy of known size.
    (None, None) when no summary exists or the kernel or its default schedule
    has changed since the counters were taken."""
    try:
        text = open(traffic_file(kernel)).read()
    except OSError:
        return None, None
    keys = ("kernel_sha256", "hbm_bytes_per_launch", "algorithmic_bytes_per_launch")
    fields = {}
    for line in text.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in keys:
            fields[k.strip()] = v.strip()
    if any(k not in fields for k in keys) or fields["kernel_sha256"] != kernel_fingerprint():
        return None, None
    return float(fields["hbm_bytes_per_launch"]), float(fields["algorithmic_bytes_per_launch"])


def _event_time(torch, stream, fn, reps):
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    e.synchronize()
    return s.elapsed_time(e) / reps


def secondary(ctx, mpc, torch, workloads, X, Y, only, cpu=True):
    ex = {}
    if "ceilings" in only:
        ex.update(ceilings())
    if "power" in only:
        ex.update(power_draw(ctx, torch, X, Y))
    if "small" in only:
        ex.update(small_latency(mpc, torch, workloads))
    if "ring_gemm" in only:
        ex.update(ring_gemm_forms(ctx, torch, X, Y))
    if "beaver_mul" in only:
        ex.update(beaver_mul_2e24(ctx, mpc, torch, X, Y))
    if "mlp" in only:
        ex.update(mlp_bench(ctx, mpc, torch, workloads))
    if "sweep" in only:
        ex["beaver_mul_sweep"] = beaver_mul_sweep(ctx, mpc, torch)
    if "multiparty" in only:
        ex.update(multiparty_bench(ctx, mpc, torch, X, Y))
    if "binary" in only:
        ex.update(binary_bench(ctx, mpc, torch, X))
    ctx.sync()
    if "grouped" in only:
        ex.update(grouped_bench(mpc, torch, workloads))
    if "grouped_schedules" in only:
        ex.update(grouped_schedules(mpc, torch, workloads))
    if "grouped_mul" in only:
        ex.update(grouped_mul_bench(mpc, torch, workloads))
    if "conv" in only:
        ex.update(conv_bench(mpc, torch, workloads, cpu))
    return ex


def power_draw(ctx, torch, X, Y):
    """Board power (hwmon power1_input, sampled every 50 ms) idle and while the
    limb GEMM of a Beaver finish (4096x4096x8192) runs back to back for 3 s,
    with its sustained rate; the board's power cap where hwmon shows it."""
    import glob
    import threading
    files = sorted(glob.glob("/sys/class/drm/card*/device/hwmon/hwmon*/power1_input"))
    if not files:
        return {}
    cap = [f.replace("power1_input", "power1_cap") for f in files]

    def read(fs):
        out = []
        for f in fs:
            try:
                out.append(int(open(f).read()) / 1e6)
            except (OSError, ValueError):
                pass
        return max(out) if out else None

    def sample(fn, secs):
        vals, on = [], [True]

        def loop():
            while on[0]:
                v = read(files)
                if v is not None:
                    vals.append(v)
                time.sleep(0.05)
        th = threading.Thread(target=loop, daemon=True)
        th.start()
        fn(secs)
        on[0] = False
        th.join()
        tail = vals[len(vals) // 3:]  # after the clock has settled
        return sum(tail) / len(tail) if tail else None

    ex = {}
    ctx.sync()
    ex["power_idle_W"] = round(sample(lambda s: time.sleep(s), 1.0), 1)
    A = torch.cat([X, X], dim=1)  # 4096 x 8192
    B = torch.cat([Y, Y], dim=0)  # 8192 x 4096
    C = ctx.empty((M, N))
    ctx.ring_gemm(A, B, "limb8", out=C)
    ctx.sync()
    ctx.profile(True)
    ctx.profile_read()

    def gemms(secs):
        t0 = time.time()
        while time.time() - t0 < secs:
            for _ in range(10):
                ctx.ring_gemm(A, B, "limb8", out=C)
            ctx.sync()
    ex["power_limb_gemm_W"] = round(sample(gemms, 3.0), 1)
    g = ctx.profile_read()["limb8"]
    ctx.profile(False)
    ex["power_limb_gemm_sustained_TOPs"] = round(72.0 * g["ring_macs"] / (g["total_ms"] * 1e-3) / 1e12, 1)
    del A, B, C
    # the MFMA-only loop of the ceilings program, back to back for 3 s
    import subprocess
    exe = os.path.join(ROOT, "paper_2109_00984_amd", "ceilings")
    res = {}

    def mfma_loop(secs):
        r = subprocess.run([exe, "mfma", str(secs)], capture_output=True, text=True, timeout=120, check=True)
        res.update(json.loads(r.stdout.strip().splitlines()[-1]))
    ex["power_mfma_loop_W"] = round(sample(mfma_loop, 3.0), 1)
    ex["power_mfma_loop_TOPs"] = res.get("mfma_i8_random_tops")
    # the vendor's int8 GEMM (torch._int_mm) on uniformly random int8, 8192^3
    a = torch.randint(-128, 128, (8192, 8192), dtype=torch.int8, device=ctx.device)
    b = torch.randint(-128, 128, (8192, 8192), dtype=torch.int8, device=ctx.device).t().contiguous().t()
    torch._int_mm(a, b)
    torch.cuda.synchronize()
    n_mm = [0]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def int_mm(secs):
        e0.record()
        t0 = time.time()
        while time.time() - t0 < secs:
            for _ in range(10):
                torch._int_mm(a, b)
            n_mm[0] += 10
            torch.cuda.synchronize()
        e1.record()
        torch.cuda.synchronize()
    ex["power_vendor_int8_gemm_W"] = round(sample(int_mm, 3.0), 1)
    ex["power_vendor_int8_gemm_TOPs"] = round(2.0 * 8192 ** 3 * n_mm[0] / (e0.elapsed_time(e1) * 1e-3) / 1e12, 1)
    del a, b
    c = read(cap)
    if c:
        ex["power_cap_W"] = round(c, 1)
    log(f"bench: power idle {ex['power_idle_W']} W, limb GEMM back to back {ex['power_limb_gemm_W']} W at "
        f"{ex['power_limb_gemm_sustained_TOPs']} TOP/s, MFMA-only loop {ex['power_mfma_loop_W']} W at "
        f"{ex['power_mfma_loop_TOPs']} TOP/s, vendor int8 GEMM {ex['power_vendor_int8_gemm_W']} W at "
        f"{ex['power_vendor_int8_gemm_TOPs']} TOP/s" + (f" (cap {ex['power_cap_W']} W)" if c else ""))
    return ex


def ceilings():
    """Sustained arithmetic ceilings measured by the library's standalone
    microbenchmark (no memory traffic): INT8 MFMA on random fragments and the
    plain form's VALU ring multiply-accumulate."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2109_00984_amd", "ceilings")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, check=True)
    c = json.loads(r.stdout.strip().splitlines()[-1])
    log(f"bench: ceilings: INT8 MFMA on random data {c['mfma_i8_random_tops']} TOP/s, "
        f"VALU ring MAC {c['valu_ring_tmacs']} T/s, HBM stream (10 in, 2 out) {c['hbm_stream_10r2w_gbs']} GB/s "
        f"at 2^24 and {c['hbm_stream_10r2w_2e28_gbs']} GB/s at 2^28 elements, HBM copy {c['hbm_copy_gbs']} GB/s")
    return {"ceiling_mfma_i8_random_TOPs": c["mfma_i8_random_tops"], "ceiling_valu_ring_TMACs": c["valu_ring_tmacs"],
            "ceiling_hbm_stream_10r2w_GBps": c["hbm_stream_10r2w_gbs"],
            "ceiling_hbm_stream_10r2w_2e28_GBps": c["hbm_stream_10r2w_2e28_gbs"],
            "ceiling_hbm_copy_GBps": c["hbm_copy_gbs"]}


def small_latency(mpc, torch, workloads):
    """The small workload: Beaver matmul X[64x128] @ W[128x32] with 2^16
    truncation (both forms) and an element-wise Beaver product over 4096
    elements; latency per call, eager and replayed from a HIP graph."""
    out = {}
    dseed = workloads.seeds(1)[2]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = mpc.Context(device=0, seed=workloads.seeds(1)[1])
        dv = lambda a: torch.from_numpy(a).to(c.device)
        x = c.share(dv(mpc.encode(workloads.uniform(1001, (64, 128), -4, 4), FRAC)), 0, 1)
        w = c.share(dv(mpc.encode(workloads.uniform(1002, (128, 32), -4, 4), FRAC)), 1, 2)
        t = c.dealer(mpc.TRIPLE_MATMUL, dseed, 3, (64, 32, 128))
        z = mpc.SharedPair(c.empty((64, 32)), c.empty((64, 32)))
        ex_ = c.share(dv(mpc.encode(workloads.uniform(1003, (4096,), -4, 4), FRAC)), 0, 4)
        ey = c.share(dv(mpc.encode(workloads.uniform(1004, (4096,), -4, 4), FRAC)), 1, 5)
        te = c.dealer(mpc.TRIPLE_MUL, dseed, 6, (4096,))
        ez = mpc.SharedPair(c.empty((4096,)), c.empty((4096,)))
        calls = {"matmul_64x128x32_plain": lambda: c.beaver_matmul(x, w, t, FRAC, "plain", out=z),
                 "matmul_64x128x32_limb8": lambda: c.beaver_matmul(x, w, t, FRAC, "limb8", out=z),
                 "matmul_64x128x32_auto": lambda: c.beaver_matmul(x, w, t, FRAC, "auto", out=z),
                 "mul_4096": lambda: c.beaver_mul(ex_, ey, te, FRAC, out=ez)}
        # what AUTO runs for this product: the launches one call adds, and
        # whether any of them is a limb GEMM
        c.sync()
        c.profile(True)
        c.profile_read()
        before = c.stats()["launches"]
        calls["matmul_64x128x32_auto"]()
        c.sync()
        launches = c.stats()["launches"] - before
        limb = c.profile_read()["limb8"]["launches"]
        c.profile(False)
        out["small_matmul_64x128x32_auto_path"] = (
            "limb8" if limb else "plain, one fused launch" if launches == 1 else f"plain, {launches} launches")
        reps = 50
        for name, fn in calls.items():
            fn()
            c.sync()
            eager = _event_time(torch, side, fn, reps)
            # one call per graph: every replay pays the runtime's graph launch
            c.graph_begin()
            fn()
            g = c.graph_end()
            c.graph_launch(g)
            c.sync()
            graph = _event_time(torch, side, lambda: c.graph_launch(g), reps)
            mpc.Context.graph_destroy(g)
            # a loop of `reps` calls captured once: what a serving loop replays
            c.graph_begin()
            for _ in range(reps):
                fn()
            g = c.graph_end()
            c.graph_launch(g)
            c.sync()
            loop = _event_time(torch, side, lambda: c.graph_launch(g), 5) / reps
            mpc.Context.graph_destroy(g)
            out[f"small_{name}_us"] = round(eager * 1e3, 2)
            out[f"small_{name}_graph_us"] = round(graph * 1e3, 2)
            out[f"small_{name}_graph_loop_us"] = round(loop * 1e3, 2)
            log(f"bench: small {name}: {eager * 1e3:.1f} us eager, {graph * 1e3:.1f} us one-call graph, "
                f"{loop * 1e3:.1f} us per call in a captured loop of {reps}")
        c.close()
    return out


def ring_gemm_forms(ctx, torch, X, Y):
    ex = {}
    # ring GEMM alone, both forms, timed with the library's launch events
    # (the fp64 limb form is the paper's method: four 16-bit limbs, ten exact
    # float64 GEMMs of the vendor BLAS; its bracket covers those GEMMs)
    C = ctx.empty((M, N))
    ctx.profile(True)
    for form, reps in (("limb8", 5), ("plain", 2), ("fp64limb", 2)):
        ctx.ring_gemm(X, Y, form, out=C)  # warm
        ctx.profile_read()
        for _ in range(reps):
            ctx.ring_gemm(X, Y, form, out=C)
        g = ctx.profile_read()[form]
        ms = g["total_ms"] / g["launches"]
        ex[f"ring_gemm_4096_{form}_tops"] = round(2.0 * M * N * K / (ms * 1e-3) / 1e12, 3)
        ex[f"ring_gemm_4096_{form}_ms"] = round(ms, 4)
        # the whole call: operand packing, the GEMM(s), the combine
        ex[f"ring_gemm_4096_{form}_call_ms"] = round(
            _event_time(torch, ctx.streams[0], lambda: ctx.ring_gemm(X, Y, form, out=C), reps), 4)
        log(f"bench: ring GEMM 4096^3 {form}: {ms:.3f} ms (call {ex[f'ring_gemm_4096_{form}_call_ms']} ms)")
    ctx.profile(False)
    ex["limb_over_plain_speedup"] = round(ex["ring_gemm_4096_plain_ms"] / ex["ring_gemm_4096_limb8_ms"], 2)
    ex["limb_over_fp64limb_speedup"] = round(ex["ring_gemm_4096_fp64limb_ms"] / ex["ring_gemm_4096_limb8_ms"], 2)
    # ten float64 multiply-adds per ring multiply-accumulate, against the FP64 matrix peak
    ex["fp64limb_gemm_fp64_frac"] = round(
        20.0 * M * N * K / (ex["ring_gemm_4096_fp64limb_ms"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)
    # the online Beaver matmul at 4096^3 over a regular and an offline-packed
    # triple (the dealer packs a1, b0, b1; the online open packs eps, a0 + eps
    # and delta only)
    import paper_2109_00984_amd as mpc
    x = ctx.share(X, 0, 91)
    y = ctx.share(Y, 1, 92)
    t = ctx.dealer(mpc.TRIPLE_MATMUL, 93, 94, (M, N, K))
    z = mpc.SharedPair(ctx.empty((M, N)), ctx.empty((M, N)))
    ex["beaver_matmul_4096_online_ms"] = round(
        _event_time(torch, ctx.streams[0], lambda: ctx.beaver_matmul(x, y, t, FRAC, "limb8", out=z), 3), 4)
    del t
    tp, packed = ctx.dealer_packed(93, 94, (M, N, K))
    ex["beaver_matmul_4096_prepacked_online_ms"] = round(
        _event_time(torch, ctx.streams[0], lambda: ctx.beaver_matmul_prepacked(x, y, tp, packed, FRAC, out=z), 3), 4)
    ex["dealer_matmul_4096_ms"] = round(
        _event_time(torch, ctx.streams[0], lambda: ctx.dealer_into(mpc.TRIPLE_MATMUL, 93, 94, (M, N, K), tp), 3), 4)
    ex["dealer_matmul_4096_packed_ms"] = round(
        _event_time(torch, ctx.streams[0], lambda: ctx._dealer_packed_into(93, 94, (M, N, K), tp, packed), 3), 4)
    # the Beaver matmul's own rate: 2 M N K ring operations over the online
    # time (open, both parties' finish, truncation), the dealer apart
    for key in ("online", "prepacked_online"):
        ex[f"beaver_matmul_4096_{key}_tops"] = round(
            2.0 * M * N * K / (ex[f"beaver_matmul_4096_{key}_ms"] * 1e-3) / 1e12, 3)
    log(f"bench: Beaver matmul 4096^3 online {ex['beaver_matmul_4096_online_ms']} ms, over a prepacked triple "
        f"{ex['beaver_matmul_4096_prepacked_online_ms']} ms; dealer {ex['dealer_matmul_4096_ms']} ms, with packing "
        f"{ex['dealer_matmul_4096_packed_ms']} ms")
    del x, y, tp, packed, z
    C0 = ctx.ring_gemm(X, Y, "limb8")
    C1 = ctx.ring_gemm(X, Y, "plain")
    C2 = ctx.ring_gemm(X, Y, "fp64limb")
    ctx.sync()
    ex["ring_gemm_forms_bit_identical"] = bool(torch.equal(C0, C1) and torch.equal(C0, C2))
    del C, C0, C1, C2
    return ex


def beaver_mul_2e24(ctx, mpc, torch, X, Y):
    ex = {}
    # Beaver element-wise product (fused mask/open/finish/truncate), HBM-bound:
    # 2^24 elements = 128 MiB per share buffer, 1.5 GiB moved per call
    n = M * K
    x = ctx.share(X.view(-1), 0, 11)
    y = ctx.share(Y.view(-1), 1, 12)
    tm = ctx.dealer(mpc.TRIPLE_MUL, 5, 13, (n,))
    zz = mpc.SharedPair(ctx.empty((n,)), ctx.empty((n,)))
    ctx.beaver_mul(x, y, tm, 16, out=zz)
    ctx.sync()
    ms = _event_time(torch, ctx.streams[0], lambda: ctx.beaver_mul(x, y, tm, 16, out=zz), 10)
    ex["beaver_mul_n"] = n
    ex["beaver_mul_ms"] = round(ms, 4)
    ex["beaver_mul_elem_per_s"] = round(n / (ms * 1e-3), 1)
    ex["beaver_mul_hbm_GBps_algorithmic"] = round(96.0 * n / (ms * 1e-3) / 1e9, 1)
    ex["beaver_mul_hbm_frac"] = round(ex["beaver_mul_hbm_GBps_algorithmic"] / HBM_PEAK_GBS, 4)
    log(f"bench: Beaver mul n=2^24: {ms:.3f} ms")
    del x, y, tm, zz
    return ex


def mlp_bench(ctx, mpc, torch, workloads):
    ex = {}
    # secure MLP 784-1024-1024-10, batch 128, square activations
    for form in ("plain", "limb8"):
        total, ops = mlp_latency(ctx, mpc, torch, workloads, form)
        ex[f"mlp_ms_{form}"] = round(total, 4)
        ex[f"mlp_graph_ms_{form}"] = round(mlp_graph_latency(mpc, torch, workloads, form), 4)
        ex[f"mlp_ops_ms_{form}"] = ops
    log(f"bench: MLP plain {ex['mlp_ms_plain']} ms, limb8 {ex['mlp_ms_limb8']} ms")
    return ex


def grouped_mul_bench(mpc, torch, workloads):
    """256 element-wise Beaver products / squares of log-uniform length in
    [2^10, 2^20] with 2^16 truncation, captured in HIP graphs and replayed:
    one grouped launch against one launch per product.  Algorithmic bytes: 96
    per product element, 64 per square."""
    rng = np.random.default_rng(workloads.seeds(6)[0])
    ns = np.exp(rng.uniform(np.log(2 ** 10), np.log(2 ** 20), 256)).astype(np.int64)
    sq = rng.random(256) < 0.25
    side = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(side):
        c = mpc.Context(device=0, seed=7)
        probs, outs = [], []
        nbytes = 0
        for i, (n, s) in enumerate(zip(ns, sq)):
            n = int(n)
            x = c.share(c.empty((n,)), 0, 3 * i)
            y = None if s else c.share(c.empty((n,)), 1, 3 * i + 1)
            t = c.dealer(mpc.TRIPLE_SQUARE if s else mpc.TRIPLE_MUL, 11, i, (n,))
            probs.append((x, y, t))
            outs.append(mpc.SharedPair(c.empty((n,)), c.empty((n,))))
            nbytes += (64 if s else 96) * n
        c.sync()

        def replay_ms(issue):
            c.graph_begin()
            issue()
            g = c.graph_end()
            c.graph_launch(g)
            c.sync()
            ms = _event_time(torch, side, lambda: c.graph_launch(g), 20)
            mpc.Context.graph_destroy(g)
            return ms

        grouped = replay_ms(lambda: c.beaver_mul_grouped(probs, FRAC, outs=outs))

        def singles():
            for (x, y, t), o in zip(probs, outs):
                c.beaver_mul(x, y, t, FRAC, out=o)

        single = replay_ms(singles)
        c.close()
    out["grouped_mul256_elements"] = int(ns.sum())
    out["grouped_mul256_graph_ms"] = round(grouped, 4)
    out["grouped_mul256_GBps_algorithmic"] = round(nbytes / (grouped * 1e-3) / 1e9, 1)
    out["grouped_mul256_one_launch_each_graph_ms"] = round(single, 4)
    log(f"bench: 256 Beaver products, graph replay: grouped {grouped:.3f} ms "
        f"({nbytes / (grouped * 1e-3) / 1e9:.0f} GB/s), one launch each {single:.3f} ms")
    return out


def grouped_bench(mpc, torch, workloads):
    """256 uneven Beaver matmuls: one open+pack launch and one GEMM launch,
    captured in a HIP graph and replayed; autotuned schedule vs the default."""
    data_seed, pseed, dseed = workloads.seeds(5)
    shapes = workloads.grouped_shapes(data_seed)
    side = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(side):
        c = mpc.Context(device=0, seed=pseed)
        probs = []
        for i, (m, n, k) in enumerate(shapes):
            x = c.share(torch.from_numpy(workloads.uniform_u64(data_seed * 1000 + 2 * i, (m, k)).view(np.int64)).to(c.device), 0, 2 * i)
            y = c.share(torch.from_numpy(workloads.uniform_u64(data_seed * 1000 + 2 * i + 1, (k, n)).view(np.int64)).to(c.device), 1, 2 * i + 1)
            probs.append((x, y, c.dealer(mpc.TRIPLE_MATMUL, dseed, i, (m, n, k))))
        outs = [mpc.SharedPair(c.empty((m, n)), c.empty((m, n))) for (m, n, k) in shapes]
        macs = float(sum(m * n * k for m, n, k in shapes))

        def timed(label, form="limb8"):
            c.beaver_matmul_grouped(probs, FRAC, form, outs=outs)  # sizes the workspace
            c.sync()
            c.graph_begin()
            c.beaver_matmul_grouped(probs, FRAC, form, outs=outs)
            g = c.graph_end()
            c.graph_launch(g)
            c.sync()
            ms = _event_time(torch, side, lambda: c.graph_launch(g), 10)
            mpc.Context.graph_destroy(g)
            out[f"grouped256_{label}_ms"] = round(ms, 4)
            out[f"grouped256_{label}_tops"] = round(2.0 * macs / (ms * 1e-3) / 1e12, 3)
            # int8 work of the finish GEMMs (2 parties x M x N x 2K ring MACs, 72 int8 ops each)
            if form == "limb8":
                out[f"grouped256_{label}_int8_frac"] = round(72.0 * 4.0 * macs / (ms * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4)
            log(f"bench: grouped 256 ({label}) graph replay {ms:.3f} ms")

        timed("plain", "plain")
        timed("default_schedule")
        # the persistent grouped launch (schedule 15, each problem in its own
        # tile class), which the autotuner below also times
        c.set_default_tile_config(15, 8, True)
        timed("persistent")
        c.set_default_tile_config(5, 8, True)
        best = c.autotune_matmul(shapes)
        out["grouped256_tuned_schedule"] = best
        timed("autotuned")
        # the same batch over offline-packed triples: the online open packs
        # eps, a0 + eps and delta only (a1, b0, b1 were packed by the dealer)
        pprobs = []
        for i, ((x, y, _), (m, n, k)) in enumerate(zip(probs, shapes)):
            t, packed = c.dealer_packed(dseed, i, (m, n, k))
            pprobs.append((x, y, t, packed))
        c.beaver_matmul_grouped_prepacked(pprobs, FRAC, outs=outs)
        c.sync()
        c.graph_begin()
        c.beaver_matmul_grouped_prepacked(pprobs, FRAC, outs=outs)
        g = c.graph_end()
        c.graph_launch(g)
        c.sync()
        ms = _event_time(torch, side, lambda: c.graph_launch(g), 10)
        mpc.Context.graph_destroy(g)
        out["grouped256_prepacked_ms"] = round(ms, 4)
        out["grouped256_prepacked_int8_frac"] = round(72.0 * 4.0 * macs / (ms * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4)
        log(f"bench: grouped 256 (autotuned, prepacked triples) graph replay {ms:.3f} ms")
        del pprobs
        out["grouped256_plaintext_macs"] = macs
        out["grouped256_limb_over_plain_speedup"] = round(out["grouped256_plain_ms"] / out["grouped256_autotuned_ms"], 2)
        out["grouped256_autotuned_over_default"] = round(
            out["grouped256_default_schedule_ms"] / out["grouped256_autotuned_ms"], 3)
        out["grouped256_autotuned_over_persistent"] = round(
            out["grouped256_persistent_ms"] / out["grouped256_autotuned_ms"], 3)
        c.close()
    return out


def grouped_schedules(mpc, torch, workloads, reps=10):
    """The 256-problem batch (plain triples) replayed from a graph under the
    one-shot classes launch (schedule 14) and the persistent one (15), each
    problem in its own tile class, `reps` replays each, for kernel traces and
    counters of the two grouped GEMM launches."""
    data_seed, pseed, dseed = workloads.seeds(5)
    shapes = workloads.grouped_shapes(data_seed)
    side = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(side):
        c = mpc.Context(device=0, seed=pseed)
        probs = []
        for i, (m, n, k) in enumerate(shapes):
            x = c.share(torch.from_numpy(workloads.uniform_u64(data_seed * 1000 + 2 * i, (m, k)).view(np.int64)).to(c.device), 0, 2 * i)
            y = c.share(torch.from_numpy(workloads.uniform_u64(data_seed * 1000 + 2 * i + 1, (k, n)).view(np.int64)).to(c.device), 1, 2 * i + 1)
            probs.append((x, y, c.dealer(mpc.TRIPLE_MATMUL, dseed, i, (m, n, k))))
        outs = [mpc.SharedPair(c.empty((m, n)), c.empty((m, n))) for (m, n, k) in shapes]
        first = None
        for sched, label in ((14, "classes"), (15, "persistent")):
            c.set_default_tile_config(sched, 8, True)
            c.beaver_matmul_grouped(probs, FRAC, "limb8", outs=outs)
            c.sync()
            got = torch.cat([torch.cat([o.s0.reshape(-1), o.s1.reshape(-1)]) for o in outs])
            first = got if first is None else first
            out["grouped256_schedules_bit_identical"] = bool(torch.equal(got, first))
            c.graph_begin()
            c.beaver_matmul_grouped(probs, FRAC, "limb8", outs=outs)
            g = c.graph_end()
            c.profile(True)
            c.profile_read()
            ms = _event_time(torch, side, lambda: c.graph_launch(g), reps)
            c.sync()
            mpc.Context.graph_destroy(g)
            # the GEMM launches alone, from the library's own event record
            # (eager: graph replays record none), one eager call per schedule
            c.beaver_matmul_grouped(probs, FRAC, "limb8", outs=outs)
            c.sync()
            gemm = c.profile_read()["limb8"]
            c.profile(False)
            out[f"grouped256_{label}_replay_ms"] = round(ms, 4)
            out[f"grouped256_{label}_gemm_ms"] = round(gemm["total_ms"] / max(1, gemm["launches"]), 4)
            log(f"bench: grouped 256 schedule {sched} ({label}): replay {ms:.3f} ms, GEMM launch "
                f"{out[f'grouped256_{label}_gemm_ms']:.3f} ms")
        c.close()
    return out


def conv_bench(mpc, torch, workloads, cpu=True):
    """The Wav2Letter-shaped conv stack (batch 8, 40x1600): 10 Beaver conv1d
    layers with truncation and 9 Beaver squares, online phase only.  With
    `cpu`, also the whole stack in the CPU oracle, checked against it."""
    data_seed, pseed, dseed = workloads.seeds(4)
    cfg = workloads.CONV
    layers = workloads.conv_shapes(cfg["batch"], cfg["length"])
    out = {}
    c = mpc.Context(device=0, seed=pseed)
    dv = lambda a: torch.from_numpy(a).to(c.device)
    X = mpc.encode(workloads.uniform(data_seed, (cfg["batch"], cfg["channels"], cfg["length"]), cfg["lo"], cfg["hi"]), FRAC)
    Xd = dv(X)
    x0 = c.share(Xd, 0, 1)
    ws, ts, ps, Wd = [], [], [], []
    for i, (b, cin, L, cout, k, s, lout) in enumerate(layers):
        W = mpc.encode(workloads.uniform(data_seed + 100 + i, (cout, cin, k), cfg["lo"], cfg["hi"]), FRAC)
        Wd.append(dv(W))
        ws.append(c.share(Wd[-1], 1, 20 + i))
        ts.append(c.dealer(mpc.TRIPLE_CONV1D, dseed, 40 + i, (b, cin, L, cout, k, s)))
        if i < len(layers) - 1:
            ps.append(c.dealer(mpc.TRIPLE_SQUARE, dseed, 60 + i, (b * cout * lout,)))
    macs = float(sum(cout * b * lout * cin * k for (b, cin, L, cout, k, s, lout) in layers))

    def forward(form):
        h = x0
        for i, (b, cin, L, cout, k, s, lout) in enumerate(layers):
            h = c.beaver_conv1d(h, ws[i], ts[i], s, FRAC, form)
            if i < len(layers) - 1:
                sq = c.beaver_mul(mpc.SharedPair(h.s0.view(-1), h.s1.view(-1)), None, ps[i], FRAC)
                h = mpc.SharedPair(sq.s0.view(b, cout, lout), sq.s1.view(b, cout, lout))
        return h

    first = None
    same = True
    # the paper's fp64 limb form too (vendor fp64 GEMMs over materialised im2col)
    for form, reps in (("limb8", 5), ("plain", 1), ("fp64limb", 1)):
        h = forward(form)
        c.sync()
        got = (h.s0.cpu().numpy().view(np.uint64), h.s1.cpu().numpy().view(np.uint64))
        if first is None:  # the limb form's output, for the oracle leg
            first = got
        same = same and all(np.array_equal(a, b) for a, b in zip(got, first))
        ms = _event_time(torch, c.streams[0], lambda: forward(form), reps)
        out[f"conv_stack_{form}_ms"] = round(ms, 3)
        out[f"conv_stack_{form}_tops"] = round(2.0 * macs / (ms * 1e-3) / 1e12, 3)
        log(f"bench: conv stack {form}: {ms:.3f} ms")
    # the CPU sample's scope on the GPU: share the input and the weights, deal
    # every triple, then the online phase (limb form), into the same buffers
    def whole():
        c.share(Xd, 0, 1, out=x0)
        for i, (b, cin, L, cout, k, s, lout) in enumerate(layers):
            c.share(Wd[i], 1, 20 + i, out=ws[i])
            c.dealer_into(mpc.TRIPLE_CONV1D, dseed, 40 + i, (b, cin, L, cout, k, s), ts[i])
            if i < len(layers) - 1:
                c.dealer_into(mpc.TRIPLE_SQUARE, dseed, 60 + i, (b * cout * lout,), ps[i])
        return forward("limb8")
    h = whole()
    c.sync()
    same = same and all(np.array_equal(a.cpu().numpy().view(np.uint64), b) for a, b in zip((h.s0, h.s1), first))
    ms = _event_time(torch, c.streams[0], whole, 3)
    out["conv_stack_limb8_with_dealer_ms"] = round(ms, 3)
    out["conv_stack_limb8_with_dealer_tops"] = round(2.0 * macs / (ms * 1e-3) / 1e12, 3)
    log(f"bench: conv stack limb8 with sharing and dealer: {ms:.3f} ms")
    out["conv_stack_forms_bit_identical"] = bool(same)
    out["conv_stack_limb_over_plain_speedup"] = round(out["conv_stack_plain_ms"] / out["conv_stack_limb8_ms"], 2)
    out["conv_stack_limb_over_fp64limb_speedup"] = round(out["conv_stack_fp64limb_ms"] / out["conv_stack_limb8_ms"], 2)
    out["conv_stack_plaintext_macs"] = macs
    c.close()
    if cpu:
        # the same seeded real inputs, encoded by the oracle itself
        Xf = workloads.uniform(data_seed, (cfg["batch"], cfg["channels"], cfg["length"]), cfg["lo"], cfg["hi"])
        Wfs = [workloads.uniform(data_seed + 100 + i, (cout, cin, k), cfg["lo"], cfg["hi"])
               for i, (b, cin, L, cout, k, s, lout) in enumerate(layers)]
        out["conv_stack_cpu_oracle"] = conv_cpu_oracle(Xf, Wfs, layers, pseed, dseed, first, macs)
    return out


def conv_cpu_oracle(Xf, Wfs, layers, pseed, dseed, want, macs):
    """The whole conv stack (all batch elements) in the CPU oracle, timed and
    checked bit for bit against the GPU's output."""
    import oracle
    t0 = time.perf_counter()
    h = oracle.share(oracle.encode(Xf, FRAC), 0, pseed, 1)
    for i, (b, cin, L, cout, k, s, lout) in enumerate(layers):
        w = oracle.share(oracle.encode(Wfs[i], FRAC), 1, pseed, 20 + i)
        h = oracle.beaver_conv1d(h, w, oracle.dealer_conv1d(dseed, 40 + i, b, cin, L, cout, k, s), s, FRAC)
        if i < len(layers) - 1:
            sq = oracle.beaver_square((h[0].ravel(), h[1].ravel()),
                                      oracle.dealer_square(dseed, 60 + i, b * cout * lout), FRAC)
            h = (sq[0].reshape(b, cout, lout), sq[1].reshape(b, cout, lout))
    dt = time.perf_counter() - t0
    ok = bool(np.array_equal(h[0], want[0]) and np.array_equal(h[1], want[1]))
    log(f"bench: conv stack cpu oracle, whole stack: {dt:.2f} s, matches the GPU: {ok}")
    return {"value": round(2.0 * macs / dt / 1e12, 6), "unit": "Tops/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": f"the whole stack at batch {layers[0][0]} (share, dealer, 10 Beaver conv1d "
                                         f"with truncation, 9 Beaver squares) in the CPU oracle; {dt:.1f} s",
            "sample_matches_gpu_bit_exact": ok}


def mlp_latency(ctx, mpc, torch, workloads, form):
    cfg = workloads.MLP
    B, dims = cfg["batch"], cfg["dims"]
    dseed = workloads.seeds(2)[2]
    X = mpc.encode(workloads.uniform(1002, (B, dims[0]), -1, 1), FRAC)
    Ws = [mpc.encode(workloads.uniform(1102 + i, (dims[i], dims[i + 1]), -1, 1), FRAC)
          for i in range(3)]
    dv = lambda a: torch.from_numpy(a).to(ctx.device)
    x = ctx.share(dv(X), 0, 100)
    ws = [ctx.share(dv(W), 1, 101 + i) for i, W in enumerate(Ws)]
    trip = [ctx.dealer(mpc.TRIPLE_MATMUL, dseed, 200 + i, (B, dims[i + 1], dims[i]))
            for i in range(3)]
    pairs = [ctx.dealer(mpc.TRIPLE_SQUARE, dseed, 300 + i, (B * dims[i + 1],)) for i in range(2)]

    def forward(keep=None):
        h = x
        for i in range(3):
            if keep is not None:
                keep.append(("matmul", i, h))
            h = ctx.beaver_matmul(h, ws[i], trip[i], FRAC, form)
            if i < 2:
                flat = mpc.SharedPair(h.s0.view(-1), h.s1.view(-1))
                if keep is not None:
                    keep.append(("square", i, flat))
                sq = ctx.beaver_mul(flat, None, pairs[i], FRAC)
                h = mpc.SharedPair(sq.s0.view(B, dims[i + 1]), sq.s1.view(B, dims[i + 1]))
        return h

    inputs = []
    forward(inputs)
    ctx.sync()
    total = _event_time(torch, ctx.streams[0], forward, 20)
    # per-operation breakdown: each op replayed alone on its recorded input
    ops = {}
    for kind, i, h in inputs:
        if kind == "matmul":
            fn = lambda h=h, i=i: ctx.beaver_matmul(h, ws[i], trip[i], FRAC, form)
            label = f"layer{i + 1}_matmul_{dims[i]}x{dims[i + 1]}"
        else:
            fn = lambda h=h, i=i: ctx.beaver_mul(h, None, pairs[i], FRAC)
            label = f"square{i + 1}_{B}x{dims[i + 1]}"
        ops[label] = round(_event_time(torch, ctx.streams[0], fn, 20), 4)
    return total, ops


def mlp_graph_latency(mpc, torch, workloads, form):
    """The same forward pass captured once in a HIP graph (outputs allocated
    up front) and replayed: the latency without host launch overhead.  Every
    replay must reproduce the eager result bit for bit."""
    cfg = workloads.MLP
    B, dims = cfg["batch"], cfg["dims"]
    dseed = workloads.seeds(2)[2]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = mpc.Context(device=0, seed=workloads.seeds(2)[1])
        dv = lambda a: torch.from_numpy(a).to(c.device)
        x = c.share(dv(mpc.encode(workloads.uniform(1002, (B, dims[0]), -1, 1), FRAC)), 0, 100)
        ws = [c.share(dv(mpc.encode(workloads.uniform(1102 + i, (dims[i], dims[i + 1]), -1, 1), FRAC)), 1, 101 + i)
              for i in range(3)]
        trip = [c.dealer(mpc.TRIPLE_MATMUL, dseed, 200 + i, (B, dims[i + 1], dims[i])) for i in range(3)]
        pairs = [c.dealer(mpc.TRIPLE_SQUARE, dseed, 300 + i, (B * dims[i + 1],)) for i in range(2)]
        hs = [mpc.SharedPair(c.empty((B, d)), c.empty((B, d))) for d in dims[1:]]
        sqs = [mpc.SharedPair(c.empty((B * d,)), c.empty((B * d,))) for d in dims[1:3]]

        def forward():
            h = x
            for i in range(3):
                h = c.beaver_matmul(h, ws[i], trip[i], FRAC, form, out=hs[i])
                if i < 2:
                    flat = mpc.SharedPair(h.s0.view(-1), h.s1.view(-1))
                    sq = c.beaver_mul(flat, None, pairs[i], FRAC, out=sqs[i])
                    h = mpc.SharedPair(sq.s0.view(B, dims[i + 1]), sq.s1.view(B, dims[i + 1]))
            return h

        out = forward()  # eager: sizes the workspace and split-K buffers
        c.sync()
        want = (out.s0.clone(), out.s1.clone())
        c.graph_begin()
        forward()
        g = c.graph_end()
        for _ in range(3):
            hs[-1].s0.zero_()
            hs[-1].s1.zero_()
            c.graph_launch(g)
            c.sync()
            assert torch.equal(hs[-1].s0, want[0]) and torch.equal(hs[-1].s1, want[1]), "graph replay differs"
        ms = _event_time(torch, side, lambda: c.graph_launch(g), 50)
        mpc.Context.graph_destroy(g)
        c.close()
    log(f"bench: MLP {form} graph replay {ms:.4f} ms")
    return ms


def multiparty_bench(ctx, mpc, torch, X, Y):
    """Three parties: the fused Beaver product and the wrap-count truncation
    (Algorithm 1) at 2^24 elements against HBM, and the Beaver matmul at
    4096^3 in the limb form (three per-party ring GEMMs of 4096x4096x8192)."""
    out = {}
    P, n = 3, 1 << 24
    x = ctx.mp_share(X.view(-1), P, 0, 90)
    y = ctx.mp_share(Y.view(-1), P, 1, 91)
    t = ctx.mp_dealer(P, mpc.TRIPLE_MUL, 17, 92, (n,))
    z = mpc.Shared([ctx.empty((n,)) for _ in range(P)])
    ctx.mp_beaver_mul(x, y, t, out=z)
    ctx.sync()
    ms = _event_time(torch, ctx.streams[0], lambda: ctx.mp_beaver_mul(x, y, t, out=z), 10)
    out["mp3_beaver_mul_ms"] = round(ms, 4)
    # 5 inputs and 1 output per party, 8 bytes each
    out["mp3_beaver_mul_GBps_algorithmic"] = round(48.0 * P * n / (ms * 1e-3) / 1e9, 1)
    r, th = ctx.mp_dealer_trunc(P, 17, 93, n)
    ctx.mp_truncate(z, 16, r, th)
    ctx.sync()
    ms = _event_time(torch, ctx.streams[0], lambda: ctx.mp_truncate(z, 16, r, th), 10)
    out["mp3_truncate_ms"] = round(ms, 4)
    # x, r, theta_r in and x out per party
    out["mp3_truncate_GBps_algorithmic"] = round(32.0 * P * n / (ms * 1e-3) / 1e9, 1)
    del t, z, r, th
    xm = mpc.Shared([v.view(M, K) for v in x])
    ym = mpc.Shared([v.view(K, N) for v in y])
    tm = ctx.mp_dealer(P, mpc.TRIPLE_MATMUL, 17, 94, (M, N, K))
    zm = mpc.Shared([ctx.empty((M, N)) for _ in range(P)])
    ctx.mp_beaver_matmul(xm, ym, tm, "limb8", out=zm)
    ctx.sync()
    ms = _event_time(torch, ctx.streams[0], lambda: ctx.mp_beaver_matmul(xm, ym, tm, "limb8", out=zm), 3)
    out["mp3_beaver_matmul_4096_ms"] = round(ms, 3)
    out["mp3_beaver_matmul_4096_tops"] = round(2.0 * M * N * K / (ms * 1e-3) / 1e12, 3)
    log(f"bench: 3 parties: Beaver mul {out['mp3_beaver_mul_GBps_algorithmic']} GB/s, truncate "
        f"{out['mp3_truncate_GBps_algorithmic']} GB/s, matmul 4096^3 {out['mp3_beaver_matmul_4096_ms']} ms")
    del x, y, tm, zm
    torch.cuda.empty_cache()
    return out


def binary_bench(ctx, mpc, torch, X):
    """Binary sharing at 2^22 words: arithmetic-to-binary conversion (7 rounds,
    12 AND triples per word) and ReLU (A2B, Algorithm 2 on the sign bit, one
    Beaver product) against HBM: each reads its shares and every triple word
    once and writes two words per element."""
    out = {}
    n = 1 << 22
    x = ctx.share(X.view(-1)[:n], 0, 95)
    t = ctx.dealer_and(19, 96, 12 * n)
    rb, ra = ctx.dealer_b2a(19, 97, n)
    tm = ctx.dealer(mpc.TRIPLE_MUL, 19, 98, (n,))
    z = mpc.SharedPair(ctx.empty((n,)), ctx.empty((n,)))
    ctx.a2b(x, 99, t, out=z)
    ctx.sync()
    ms = _event_time(torch, ctx.streams[0], lambda: ctx.a2b(x, 99, t, out=z), 10)
    out["a2b_2^22_ms"] = round(ms, 4)
    out["a2b_GBps_algorithmic"] = round(8.0 * (2 + 72 + 2) * n / (ms * 1e-3) / 1e9, 1)
    ctx.relu(x, 99, t, rb, ra, tm, out=z)
    ctx.sync()
    ms = _event_time(torch, ctx.streams[0], lambda: ctx.relu(x, 99, t, rb, ra, tm, out=z), 10)
    out["relu_2^22_ms"] = round(ms, 4)
    out["relu_GBps_algorithmic"] = round(8.0 * (2 + 72 + 4 + 6 + 2) * n / (ms * 1e-3) / 1e9, 1)
    log(f"bench: binary: A2B 2^22 {out['a2b_2^22_ms']} ms ({out['a2b_GBps_algorithmic']} GB/s), ReLU "
        f"{out['relu_2^22_ms']} ms ({out['relu_GBps_algorithmic']} GB/s)")
    del x, t, rb, ra, tm, z
    torch.cuda.empty_cache()
    return out


def beaver_mul_sweep(ctx, mpc, torch):
    """Beaver element-wise product (mask, open, finish, 2^16 truncation in one
    pass) from 2^12 to 2^28 elements: algorithmic GB/s at 96 B per element."""
    out = {}
    dev = ctx.device
    for lg in range(12, 29, 2):
        n = 1 << lg
        g = torch.Generator(device=dev)
        g.manual_seed(lg)
        X = torch.randint(-(1 << 62), 1 << 62, (n,), device=dev, generator=g, dtype=torch.int64)
        Y = torch.randint(-(1 << 62), 1 << 62, (n,), device=dev, generator=g, dtype=torch.int64)
        x = ctx.share(X, 0, 70 + lg)
        y = ctx.share(Y, 1, 71 + lg)
        del X, Y
        t = ctx.dealer(mpc.TRIPLE_MUL, 9, 72 + lg, (n,))
        z = mpc.SharedPair(ctx.empty((n,)), ctx.empty((n,)))
        ctx.beaver_mul(x, y, t, FRAC, out=z)
        ctx.sync()
        reps = max(3, min(200, (1 << 26) // n))
        ms = _event_time(torch, ctx.streams[0], lambda: ctx.beaver_mul(x, y, t, FRAC, out=z), reps)
        out[f"2^{lg}"] = {"us": round(ms * 1e3, 2), "elem_per_s": round(n / (ms * 1e-3), 1),
                          "GBps": round(96.0 * n / (ms * 1e-3) / 1e9, 1)}
        del x, y, t, z
        torch.cuda.empty_cache()
    log("bench: Beaver mul sweep " + ", ".join(f"{k}: {v['GBps']} GB/s" for k, v in out.items()))
    return out


def cpu_baseline(Xh, Yh, party_seed, dealer_seed, z_rows):
    """The CPU oracle on the first `rows` rows of the same workload (row slices of
    a row-major PRG fill are the same draws as in the full problem)."""
    import oracle

    def run(rows):
        t0 = time.perf_counter()
        xs = oracle.share(Xh[:rows], 0, party_seed, 1)
        ys = oracle.share(Yh, 1, party_seed, 2)
        tr = oracle.dealer_matmul(dealer_seed, 3, rows, N, K)
        zz = oracle.beaver_matmul(xs, ys, tr, FRAC)
        oracle.reveal(*zz)
        return time.perf_counter() - t0, zz

    # calibrate on 64 rows, then aim at about 15 s of oracle work (at most the
    # whole 4096-row step); the operand-B share and triple are a fixed cost, so
    # the row count is re-estimated once more if the first estimate falls short
    rows = 64
    dt, zz = run(rows)
    log(f"bench: cpu oracle {rows} rows: {dt:.2f} s")
    for _ in range(2):
        if dt >= 10.0 or rows >= M:
            break
        rows = int(min(M, max(rows + 64, rows * 15.0 / dt)))
        rows -= rows % 64
        dt, zz = run(rows)
        log(f"bench: cpu oracle {rows} rows: {dt:.2f} s")
    match = bool(np.array_equal(zz[0], z_rows[0][:rows]) and np.array_equal(zz[1], z_rows[1][:rows]))
    cores = oracle.num_threads()
    # the paper's CPU setting: one thread, on a smaller slice
    oracle.set_num_threads(1)
    rows1 = 16
    dt1, zz1 = run(rows1)
    oracle.set_num_threads(cores)
    log(f"bench: cpu oracle 1 thread, {rows1} rows: {dt1:.2f} s")
    match = match and bool(np.array_equal(zz1[0], z_rows[0][:rows1]))
    return {"value": round(2.0 * rows * N * K / dt / 1e12, 6), "unit": "Tops/s",
            "cores": cores, "kind": "oracle",
            "sample": f"rows 0..{rows - 1} of the 4096^3 step (share, dealer, Beaver matmul, "
                      f"truncate, reveal) in the CPU oracle; {dt:.1f} s",
            "sample_matches_gpu_bit_exact": match,
            "one_thread": {"value": round(2.0 * rows1 * N * K / dt1 / 1e12, 6),
                           "unit": "Tops/s", "cores": 1,
                           "sample": f"rows 0..{rows1 - 1}; {dt1:.1f} s"}}

if __name__ == "__main__":
    sys.exit(main())
