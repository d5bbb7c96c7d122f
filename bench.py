#!/usr/bin/env python3
"""Throughput of the NSHEDB equality mask on one MI355X.

One step = EQ(x, y) = 1 - (x - y)^(p-1) (Eq. eq:equality) over one column
of 2^20 rows held as 32 BFV ciphertexts of 32,768 slots (n = 32768,
log2(Q*P) <= 881, p = 65537: Sec. 5.1), i.e. the subtraction, 16 squarings
each with relinearization, and the negate-and-add - every step of the hot
path - with inputs already resident in HBM.  value = records (slots) per
second.  The line also carries:

  roofline      the dominant kernel's algorithmic FP64 VALU work per launch
                over its mean launch time (HIP events on the launch stream,
                recorded around every launch inside the timed region), against
                the chip's FP64 VALU issue peak;
  kernels       per-kernel-kind time and launch counts from the same events;
  roofline_ks_mac  the key-switch product's algorithmic HBM bytes per launch
                over its mean launch time, against the 8 TB/s HBM peak;
  rates         squarings/s, transformed residues/s, modular products/s;
  latency_1ct_ms  one ciphertext (32,768 rows) through the whole mask;
  batched       512 instances of uneven size (rows log-uniform in
                [2^14, 2^20]) in HIP-graph waves (autotuned launch shapes and
                wave size) vs a per-instance launch loop;
  batched_128   the same for 128 instances, rows in [2^16, 2^20];
  next_rows     IN against 4 members, SELECT, the rotate-and-add SUM/COUNT,
                LT against a constant and a 4-row JOIN over the same column;
  cpu_baseline  the exact-integer oracle on a bounded sample, host cores.

Inputs are seeded uniform residues: a fresh RLWE ciphertext is uniform to
anyone without the key, and every kernel is data-oblivious.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (= 78.6 TFLOP/s counting an FMA as two flops).
PEAK_FP64_OPS = 256 * 64 * 2.4e9
# Algorithmic FP64 VALU operations of one exact modular butterfly: the
# modular product (mul, fma, mul, rndne, fma, add = 6, the error-free FMA
# formulation) and the sum and difference (2).  Range reductions the
# kernel adds (lazy, once per round) are overhead, not counted.
OPS_PER_BUTTERFLY = 8
PAPER_RECORDS_PER_S = 1.0 / 0.09e-3   # 0.09 ms per record, 1 CPU thread (SEAL)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the built library (its machine code): HBM counters taken on
    one build are reported only while the library is bit-identical (the
    build compiles in a fixed directory, so the same sources rebuild to the
    same bytes)."""
    lib = os.path.join(ROOT, "paper_2602_24271_amd", "libnshe.so")
    if not os.path.exists(lib):
        return "none"
    h = hashlib.sha256()
    with open(lib, "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


# A digit's value in a target prime from its alpha mixed-radix digits,
# v_0 + [q_g]_p v_1 (+ [q_g q_g+1]_p v_2): alpha - 1 exact modular products
# (6 FP64 operations each) and as many additions per coefficient
OPS_PER_MODUP = 7


# One term y M of a base-conversion row, computed exactly as four FMAs on
# 24-bit halves (y = y_h 2^24 + y_l, M = c1 2^24 + c0).
OPS_PER_CONV_TERM = 4


def _traffic(kind: str):
    """HBM bytes per launch of a kernel kind from profiles/traffic.json, while
    the built library is the profiled one."""
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tf):
        return None
    with open(tf) as fh:
        t = json.load(fh)
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch", {}).get(kind)


def roofline_scale(prof: dict, ctx) -> dict | None:
    """The scale-and-round (FP64 VALU): per coefficient of the tensor product
    (three per ciphertext coefficient) two exact base conversions, L -> L + 1
    and L + 1 -> L primes, L (L + 1) terms each at OPS_PER_CONV_TERM FP64
    operations; its reductions, modular products and the digits' mixed-radix
    digits are overhead."""
    st = prof.get("scale")
    if not st or not st["launches"] or ctx is None:
        return None
    coeffs = st["work"] / st["launches"]
    ops = coeffs * 2 * ctx.L * ctx.L_ext * OPS_PER_CONV_TERM
    avg_s = st["ms"] / st["launches"] / 1e3
    return {"bound": "alu", "kernel": "scale", "achieved": ops / avg_s / 1e12,
            "peak": PEAK_FP64_OPS / 1e12, "unit": "TOP/s (FP64 VALU ops)",
            "frac": ops / avg_s / PEAK_FP64_OPS, "traffic": _traffic("scale"),
            "coefficients_per_launch": coeffs, "ops_per_launch": ops,
            "mean_launch_ms": st["ms"] / st["launches"]}


def roofline_dominant(prof: dict, ctx) -> tuple[dict, dict]:
    """The roofline of the kernel kind with the most time (the scale-and-round
    or a transform), and the heaviest transform's."""
    ntt, _ = roofline(prof, ctx)
    dom = max(prof, key=lambda k: prof[k]["ms"])
    if dom == "scale":
        sc = roofline_scale(prof, ctx)
        if sc is not None:
            sc["dominant_kind"] = dom
            return sc, ntt
    return ntt, ntt


def roofline(prof: dict, ctx=None) -> tuple[dict, str]:
    ntt = {k: v for k, v in prof.items() if k.startswith("ntt")}
    dom = max(prof, key=lambda k: prof[k]["ms"])
    if dom not in ntt:
        # report the heaviest transform kind; the dominant kind is named too
        dom_ntt = max(ntt, key=lambda k: ntt[k]["ms"])
    else:
        dom_ntt = dom
    st = prof[dom_ntt]
    per_launch_ops = st["work"] / st["launches"] * OPS_PER_BUTTERFLY
    modup = 0.0
    stages = None
    if ctx is not None and dom_ntt == "ntt_digit":
        n = ctx.n
        stages = n.bit_length() - 1
        if n == 1 << 15 and ctx.tuning()["split_forward"]:
            # by coefficient parity: two 2^14-point transforms per limb, the
            # last stage left to the key-switch product
            stages -= 1
    if stages and getattr(ctx, "alpha", 1) > 1:
        # digits of alpha primes: each limb transform first forms the digit's
        # value in its prime (N coefficients, alpha - 1 products and adds each)
        limbs = st["work"] / st["launches"] / (n // 2 * stages)
        modup = limbs * n * OPS_PER_MODUP * (ctx.alpha - 1)
        per_launch_ops += modup
    avg_s = st["ms"] / st["launches"] / 1e3
    achieved = per_launch_ops / avg_s
    traffic = _traffic(dom_ntt)
    return {
        "bound": "alu",
        "kernel": dom_ntt,
        "dominant_kind": dom,
        "achieved": achieved / 1e12,
        "peak": PEAK_FP64_OPS / 1e12,
        "unit": "TOP/s (FP64 VALU ops)",
        "frac": achieved / PEAK_FP64_OPS,
        "traffic": traffic,
        "butterflies_per_launch": st["work"] / st["launches"],
        "stages_per_limb": stages,
        "modup_ops_per_launch": modup,
        "mean_launch_ms": st["ms"] / st["launches"],
    }, dom_ntt


PEAK_HBM_BYTES = 8.0e12   # MI355X HBM3E


def roofline_ks(ctx, prof: dict, n_ct: int, ks_chunk: int) -> dict | None:
    """The key-switch product (HBM-bound), against the HBM peak: per launch it
    reads the n_ct ciphertexts' digits (dnum digits x (L+alpha) limbs x N
    doubles each), the key (dnum x 2 x (L+alpha) x N) once per chunk of
    ks_chunk ciphertexts, and writes 2 x (L+alpha) x N sums per ciphertext."""
    st = prof.get("ks_mac")
    if not st or not st["launches"]:
        return None
    n, D, K = ctx.n, ctx.dnum, ctx.L + ctx.alpha
    # the launcher's chunk: halved down to the ciphertexts present, and at
    # most 16 with digit transforms by parity (four sums per ciphertext)
    while ks_chunk > 4 and ks_chunk // 2 >= n_ct:
        ks_chunk //= 2
    if n == 1 << 15 and ctx.tuning()["split_forward"]:
        ks_chunk = min(ks_chunk, 16)
    chunks = -(-n_ct // ks_chunk)
    per_launch = 8 * n * K * (n_ct * D + chunks * 2 * D + n_ct * 2)
    avg_s = st["ms"] / st["launches"] / 1e3
    return {"bound": "hbm", "kernel": "ks_mac", "achieved": per_launch / avg_s / 1e9,
            "peak": PEAK_HBM_BYTES / 1e9, "unit": "GB/s", "frac": per_launch / avg_s / PEAK_HBM_BYTES,
            "bytes_per_launch": per_launch, "mean_launch_ms": st["ms"] / st["launches"]}


def _host_cpu() -> str:
    cpu = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return cpu


# The CPU phase runs before anything touches the GPU: its process pool is
# forked from a process that holds no device state.
_POOL = {}


def _pool_square(k: int) -> tuple[float, float]:
    """One worker: encrypt ciphertext k of the 2^20-row column pair (seed 0;
    setup, untimed), then one squaring with relinearization of x_k - y_k,
    timed.  Returns (seconds, setup seconds)."""
    import synth
    from oracle import bfv
    pr, sk, rk = _POOL["pr"], _POOL["sk"], _POOL["rk"]
    n = pr.n
    t0 = time.perf_counter()
    x, y = synth.column_pair_half_match(0, 32 * n)
    sl = slice(k * n, (k + 1) * n)
    cx = bfv.encrypt_slots(pr, sk, x[sl], synth.enc_randomness(1000 + k, n, pr.q))
    cy = bfv.encrypt_slots(pr, sk, y[sl], synth.enc_randomness(2000 + k, n, pr.q))
    z = bfv.sub(pr, cx, cy)
    t1 = time.perf_counter()
    bfv.square_relin(pr, rk, z)
    return time.perf_counter() - t1, t1 - t0


def _pool_encrypt(i: int):
    """Encryptions for the batched leg's decrypt check: instance i is one
    32,768-row ciphertext of sorted dictionary ids (seed 100 + i) against
    one encrypted id of the dictionary."""
    import synth
    from oracle import bfv
    pr, sk = _POOL["pr"], _POOL["sk"]
    n = pr.n
    x, y = synth.column_structured(100 + i, n)
    cx = bfv.encrypt_slots(pr, sk, x, synth.enc_randomness(5000 + i, n, pr.q))
    cy = bfv.encrypt_slots(pr, sk, y, synth.enc_randomness(6000 + i, n, pr.q))
    return x, int(y[0]), np.stack([bfv.to_limbs(c, pr.q) for c in cx]), \
        np.stack([bfv.to_limbs(c, pr.q) for c in cy])


def cpu_phase(full_chain: bool, alpha: int = 1) -> dict:
    """The exact-integer oracle (untuned) on the host cores, on bounded
    samples of the workload:
      * the whole EQ (16 levels) of one N = 1024 ciphertext pair (seed 0),
        one core;
      * one squaring with relinearization (1/16 of a ciphertext's EQ) of
        each of C ciphertexts of the 2^20-row column, one per worker of a
        pool of C processes (C = the host cores given to this process, at
        most 16): rate = C x 32768 records / (16 x the pool's wall time);
      * with full_chain, one 32,768-slot ciphertext's whole EQ on one core.
    Also encrypts the inputs of the batched decrypt check and returns the
    key it used."""
    import multiprocessing as mp
    import synth
    from oracle import bfv
    out = {}
    # N = 1024, the whole chain
    n0 = 1024
    pr0 = bfv.paper_params(n0, alpha=alpha)
    sk0, rk0 = bfv.keygen(pr0, synth.key_randomness(0, n0, pr0.moduli_pq, pr0.dnum))
    x0, y0 = synth.column_pair_half_match(0, n0)
    c0x = bfv.encrypt_slots(pr0, sk0, x0, synth.enc_randomness(1, n0, pr0.q))
    c0y = bfv.encrypt_slots(pr0, sk0, y0, synth.enc_randomness(2, n0, pr0.q))
    t0 = time.perf_counter()
    bfv.eq_chain(pr0, rk0, c0x, c0y)
    t_small = time.perf_counter() - t0
    out["n1024_chain"] = {"seconds": t_small, "records_per_s": n0 / t_small, "cores": 1}
    log(f"oracle: N=1024 EQ chain {t_small:.2f} s")
    # N = 32768: keys (and the key's transform into the oracle's basis) once,
    # shared by the forked workers
    n = 32768
    pr = bfv.paper_params(n, alpha=alpha)
    t0 = time.perf_counter()
    sk, rk = bfv.keygen(pr, synth.key_randomness(0, n, pr.moduli_pq, pr.dnum))
    bfv.prepare_key(pr, rk)
    log(f"oracle: keys at N=32768 {time.perf_counter() - t0:.1f} s")
    _POOL.update(pr=pr, sk=sk, rk=rk)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(16, avail))
    with mp.get_context("fork").Pool(cores) as pool:
        t0 = time.perf_counter()
        res = pool.map(_pool_square, range(cores))
        wall = time.perf_counter() - t0
        setup = max(r[1] for r in res)
        check = pool.map(_pool_encrypt, range(8))
    sq = [r[0] for r in res]
    # the pool's wall time minus the encryptions each worker did first
    t_level = max(sq)
    out["pool"] = {"cores": cores, "squaring_seconds": sq, "wall_seconds": wall,
                   "setup_seconds_max": setup}
    out["value"] = cores * n / (16 * t_level)
    out["single_core_records_per_s"] = n / (16 * (sum(sq) / len(sq)))
    log(f"oracle: {cores} workers, one squaring each, {t_level:.2f} s (wall {wall:.1f} s)")
    if full_chain:
        x, y = synth.column_pair_half_match(0, 32 * n)
        cx = bfv.encrypt_slots(pr, sk, x[:n], synth.enc_randomness(1000, n, pr.q))
        cy = bfv.encrypt_slots(pr, sk, y[:n], synth.enc_randomness(2000, n, pr.q))
        t0 = time.perf_counter()
        bfv.eq_chain(pr, rk, cx, cy)
        t_full = time.perf_counter() - t0
        out["n32768_chain"] = {"seconds": t_full, "records_per_s": n / t_full, "cores": 1}
        log(f"oracle: N=32768 EQ chain {t_full:.1f} s")
    out["check"] = check
    out["keys"] = (pr, sk, rk)
    return out


def cpu_baseline(cp: dict) -> dict:
    return {"value": cp["value"], "unit": "records/s", "cores": cp["pool"]["cores"],
            "kind": "oracle",
            "sample": (f"one squaring + relinearization (1/16 of the EQ) of each of "
                       f"{cp['pool']['cores']} ciphertexts of the 2^20-row column, one per "
                       f"process, x16; inputs encrypted first (untimed)"),
            "single_core_records_per_s": cp["single_core_records_per_s"],
            "pool": cp["pool"], "n1024_chain": cp["n1024_chain"],
            "n32768_chain": cp.get("n32768_chain"),
            "host_cpu": _host_cpu(), "host_cores_available": os.cpu_count()}


def batched_check(cp: dict, wave: int, alpha: int = 1) -> dict:
    """A seeded oracle sample of the batched workload: 8 one-ciphertext
    instances (real encryptions with the oracle's key) through the batched
    call in graph waves; every mask decrypts to [x == c]."""
    import torch
    from oracle import bfv
    from paper_2602_24271_amd import Context
    pr, sk, rk = cp["keys"]
    ctx = Context.paper(15, alpha=alpha)
    ctx.set_relin_key(torch.from_numpy(rk.limbs(pr)).to(ctx.device))
    items = [(torch.from_numpy(cx[None]).to(ctx.device), torch.from_numpy(cy[None]).to(ctx.device))
             for _, _, cx, cy in cp["check"]]
    outs = ctx.eq_mask_batched(items, wave_ct=wave, use_graph=True)
    torch.cuda.synchronize()
    ok = 0
    for (x, c, _, _), o in zip(cp["check"], outs):
        a = o[0].cpu().numpy()
        ct = tuple(bfv.from_limbs(a[k], pr.q) for k in range(2))
        ok += int(list(bfv.decrypt_slots(pr, sk, ct)) == list((x == c).astype(int)))
    ctx.close()
    log(f"batched decrypt check: {ok} of {len(items)} masks decrypt to [x == c]")
    return {"instances": len(items), "ciphertexts": len(items), "wave_ct": wave,
            "masks_decrypting_correctly": ok}


def probes(ctx) -> dict:
    """The ceilings: the exact modular product's chip-wide rate, whether FP64
    MFMA adds FP64 throughput to the VALU, and one base conversion (17 -> 18
    primes over the scale-and-round's 3 x 2^20 coefficients) by split-FMA
    rows and by integer MFMA."""
    import ctypes
    from paper_2602_24271_amd import _lib
    lib = _lib.load()
    m = _lib.NsheModmulProbe()
    _lib.check(lib.nshe_probe_modmul(0, 4096, ctypes.byref(m)))
    out = {"modmul": {"products_per_s": m.products_per_s, "fp64_ops_per_s": m.fp64_ops_per_s,
                      "frac_of_issue_peak": m.fp64_ops_per_s / PEAK_FP64_OPS}}
    ov = _lib.NsheOverlapProbe()
    _lib.check(lib.nshe_probe_fp64_overlap(0, 2000, ctypes.byref(ov)))
    out["fp64_mfma_overlap"] = {"ms_valu": ov.ms_valu, "ms_mfma": ov.ms_mfma, "ms_both": ov.ms_both,
                                "fma_per_s_valu": ov.fma_per_s_valu,
                                "fma_per_s_mfma": ov.fma_per_s_mfma}
    # the probe is built for 17 -> 18 primes: the one-special-prime basis
    from paper_2602_24271_amd import Context
    c17 = ctx if ctx.L == 17 else Context.paper(15)
    qin = (ctypes.c_uint64 * c17.L)(*c17.q)
    qout = (ctypes.c_uint64 * c17.L_ext)(*c17.ext_primes)
    r = _lib.NsheConvProbe()
    n = 3 << 20
    _lib.check(lib.nshe_probe_conversion(0, qin, c17.L, qout, c17.L_ext, n, 5, ctypes.byref(r)))
    out["conversion_17_to_18"] = {"coefficients": n, "ms_split_fma": r.ms_fma,
                                  "ms_mfma_i8": r.ms_mfma, "mismatches": r.mismatches}
    if c17 is not ctx:
        c17.close()
    log(f"probes: FP64 VALU {ov.ms_valu:.2f} ms, MFMA {ov.ms_mfma:.2f} ms, both {ov.ms_both:.2f} ms")
    log(f"probes: modmul {m.fp64_ops_per_s / 1e12:.1f} T FP64 ops/s; conversion fma "
        f"{r.ms_fma:.3f} ms, mfma {r.ms_mfma:.3f} ms, mismatches {r.mismatches}")
    return out


def batched(ctx, n_inst: int, reps: int, max_wave: int = 128, seed: int = 2,
            lo_rows: int = 1 << 14, hi_rows: int = 1 << 20) -> dict:
    """n_inst instances with rows log-uniform in [lo_rows, hi_rows] (one
    encrypted constant each as y), HIP-graph waves vs a per-instance loop."""
    import torch
    import synth
    rows = synth.log_uniform_sizes(seed, n_inst, lo_rows, hi_rows)
    cts = [int(math.ceil(r / ctx.n)) for r in rows]
    total = sum(cts)
    dev = ctx.device
    items = []
    for i, m in enumerate(cts):
        x = synth.uniform_device_residues((m, 2), ctx.q, ctx.n, 1000 * seed + 10000 + i, dev)
        y = synth.uniform_device_residues((1, 2), ctx.q, ctx.n, 1000 * seed + 50000 + i, dev)
        items.append((x, y))
    outs = [torch.empty_like(x) for x, _ in items]
    # autotune launch shapes and the wave size on the largest instance
    sample = max(items, key=lambda it: it[0].shape[0])[0]
    t0 = time.perf_counter()
    tuned = ctx.autotune(sample, max_wave_ct=max_wave)
    t_tune = time.perf_counter() - t0
    wave = tuned["wave_ct"]
    log(f"autotuned in {t_tune:.1f} s: {tuned}")
    log(f"batched: {n_inst} instances, {total} ciphertexts, wave {wave}")
    # graph path
    ctx.eq_mask_batched(items, wave_ct=wave, use_graph=True, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.eq_mask_batched(items, wave_ct=wave, use_graph=True, outs=outs)
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    log(f"batched graph {t_graph * 1e3:.1f} ms")
    # per-instance loop
    for (x, y), o in zip(items[:4], outs[:4]):
        ctx.eq_mask(x, y, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for (x, y), o in zip(items, outs):
            ctx.eq_mask(x, y, o)
    torch.cuda.synchronize()
    t_loop = (time.perf_counter() - t0) / reps
    log(f"per-instance loop {t_loop * 1e3:.1f} ms")
    recs = total * ctx.n
    return {"instances": n_inst, "rows_range": [lo_rows, hi_rows], "seed": seed,
            "ciphertexts": total, "wave_ct": wave,
            "autotuned": tuned, "autotune_s": t_tune,
            "records_per_s_graph": recs / t_graph, "records_per_s_loop": recs / t_loop,
            "ms_graph": t_graph * 1e3, "ms_loop": t_loop * 1e3, "speedup": t_loop / t_graph}


def derived_rates(ctx, prof: dict, steps: int, n_ct: int, ms: float) -> dict:
    """The timed steps in the method's own units per second: squarings (one
    per ciphertext and level), residues through a number-theoretic transform
    (forward or inverse; from the transform launches' butterfly counts) and
    algorithmic modular products.  Products per ciphertext and level, with
    L data primes, LB = L + 1 extension primes and N coefficients: one per
    butterfly; the squaring's tensor 3 (L + LB) N; the lift 2 (L + LB L) N;
    the scale-and-round 3 (L + LB (L + 1) + L LB) N; the key-switch inner
    product 2 D (L + A) N with D digits of A primes; the mod-down
    2 ((1 + A) L + A) N; with A = 2 also the digits' mixed radix (L / 2) N
    and their values in every target prime D (L + A) N."""
    sec = ms / 1e3
    n, L, A, D = ctx.n, ctx.L, ctx.alpha, ctx.dnum
    LB = L + 1
    log2n = n.bit_length() - 1
    bfly = sum(v["work"] for k, v in prof.items() if k.startswith("ntt")) / steps
    levels = ctx.squarings * n_ct
    per_level = (3 * (L + LB) + 2 * (L + LB * L) + 3 * (L + LB * (L + 1) + L * LB)
                 + 2 * D * (L + A) + 2 * ((1 + A) * L + A)
                 + ((L // 2 + D * (L + A)) if A == 2 else 0)) * n
    return {"squarings_per_s": levels / sec,
            "ntt_residues_per_s": bfly * 2 / log2n / sec,
            "modmul_per_s": (bfly + levels * per_level) / sec,
            "modmul_per_step": bfly + levels * per_level}


def eq_setup(alpha: int, n_ct: int, ks_fused: int, dev, streams: int = 0):
    """A paper-parameter context with alpha special primes, a uniform
    stand-in relinearization key and a seeded uniform column pair of n_ct
    ciphertexts (seeds 0 and 1; timing is data-oblivious)."""
    import torch
    import synth
    from paper_2602_24271_amd import Context
    ctx = Context.paper(15, alpha=alpha)
    if ks_fused in (0, 1):
        ctx.set_tuning(ks_fused=ks_fused)
    if streams in (1, 2):
        ctx.set_tuning(streams=streams)
    log(f"context N={ctx.n} L={ctx.L}+{ctx.alpha} ext={ctx.L_ext} squarings={ctx.squarings}")
    x = synth.uniform_device_residues((n_ct, 2), ctx.q, ctx.n, 0, dev)
    y = synth.uniform_device_residues((n_ct, 2), ctx.q, ctx.n, 1, dev)
    evk = synth.uniform_device_residues((ctx.dnum, 2), ctx.moduli_pq, ctx.n, 2, dev)
    ctx.set_relin_key(evk)
    del evk
    out = torch.empty_like(x)
    ctx.workspace(n_ct)
    return ctx, x, y, out


def step_ms(ctx, x, y, out, steps: int) -> float:
    """Mean time of `steps` EQ calls (HIP events on the current stream,
    which every call joins back to)."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        ctx.eq_mask(x, y, out)
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def eq_steps(ctx, x, y, out, steps: int, warmup: int):
    """warmup untimed EQ steps, then `steps` timed ones in the context's
    schedule (with the tuning's two streams: the column's halves on two
    streams), then `steps` more with every launch timed (profiling runs each
    call on one stream, so a launch's time is its own, on the whole GPU):
    (ms per step, profile, exact-lift fallbacks taken, ms per step on one
    stream or None when the schedule is one stream)."""
    import torch
    ctx.reset_margin_events()
    for _ in range(warmup):
        ctx.eq_mask(x, y, out)
    torch.cuda.synchronize()
    log("warmup done")
    ms = step_ms(ctx, x, y, out, steps)
    ms_one = None
    if ctx.tuning()["streams"] == 2 and x.shape[0] >= 32:
        ctx.set_tuning(streams=1)
        ctx.eq_mask(x, y, out)
        ms_one = step_ms(ctx, x, y, out, steps)
        ctx.set_tuning(streams=2)
    ctx.profile(True)
    for _ in range(steps):
        ctx.eq_mask(x, y, out)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    return ms, prof, ctx.margin_events(), ms_one


def timed(fn, reps: int) -> float:
    """Mean wall time (s) of fn() over reps calls after one untimed call,
    the device synchronised around the timed region."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def next_rows(ctx, x, mask, reps: int) -> dict:
    """The operators built on EQ over the same column (n_ct ciphertexts):
    IN against 4 encrypted members (Eq. eq:in), SELECT (Eq. eq:select), the
    rotate-and-add SUM/COUNT (Sec. 4.2.2) with 15 Galois keys, and LT against
    one constant (Eq. eq:inequality).  Keys, members and the constant are
    seeded uniform residues (timing is data-oblivious)."""
    import synth
    dev = ctx.device
    n_ct = x.shape[0]
    rows = n_ct * ctx.n
    out = {}
    k = 4
    members = synth.uniform_device_residues((k, 2), ctx.q, ctx.n, 30, dev)
    t = timed(lambda: ctx.in_mask(x, members), reps)
    out["in"] = {"members": k, "rows": rows, "ms": t * 1e3, "records_per_s": rows / t,
                 "eq_records_per_s": k * rows / t,
                 "paper_ms_per_record": 0.09, "paper_source": "Table tab:primitive-times, IN row"}
    log(f"IN (k={k}) {t * 1e3:.1f} ms")
    t = timed(lambda: ctx.select(x, mask), reps)
    out["select"] = {"rows": rows, "ms": t * 1e3, "records_per_s": rows / t}
    log(f"SELECT {t * 1e3:.2f} ms")
    key = synth.uniform_device_residues((ctx.dnum, 2), ctx.moduli_pq, ctx.n, 31, dev)
    els = ctx.galois_elements()
    for g in els:
        ctx.set_galois_key(g, key)
    del key
    sel = ctx.select(x, mask)
    t = timed(lambda: ctx.sum_slots(sel), reps)
    ctx.profile(True)                 # one more call, every launch timed
    ctx.sum_slots(sel)
    prof = ctx.profile_read()
    ctx.profile(False)
    roof, _ = roofline(prof, ctx)
    out["sum_slots"] = {"rotations": len(els), "rows": rows, "ms": t * 1e3,
                        "records_per_s": rows / t, "roofline": roof,
                        "kernels": {kk: {"launches": v["launches"], "ms": v["ms"]}
                                    for kk, v in prof.items()},
                        "paper_ms_per_record": 0.04,
                        "paper_source": "Table tab:primitive-times, SUM and COUNT rows"}
    log(f"SUM/COUNT ({len(els)} rotations) {t * 1e3:.1f} ms")
    # LT against a broadcast constant, in chunks of 16 ciphertexts (the
    # comparison workspace holds about 420 ciphertext arrays per chunk: 56 GB
    # for 16 at N = 32768; chunks of 8 took 8% longer, of 32 3% less, with 111 GB)
    const = synth.uniform_device_residues((1, 2), ctx.q, ctx.n, 32, dev)
    chunk = min(16, n_ct)

    def lt_column():
        for c0 in range(0, n_ct, chunk):
            ctx.compare(x[c0:c0 + chunk], const, "lt")

    ctx.compare(x[:chunk], const, "lt")
    t = timed(lt_column, 1)
    ctx.profile(True)                 # one chunk, every launch timed
    ctx.compare(x[:chunk], const, "lt")
    prof = ctx.profile_read()
    ctx.profile(False)
    roof, _ = roofline(prof, ctx)
    out["lt"] = {"rows": rows, "chunk_ct": chunk, "ms": t * 1e3, "records_per_s": rows / t,
                 "roofline": roof,
                 "kernels": {kk: {"launches": v["launches"], "ms": v["ms"]}
                             for kk, v in prof.items()},
                 "paper_ms_per_record": 3.66,
                 "paper_source": "Table tab:primitive-times, Comparison rows"}
    log(f"LT {t * 1e3:.1f} ms")
    # JOIN: the column as fact-table keys against 4 rows of one reference
    # ciphertext (keys and an attribute), Galois keys as loaded above
    b_key = synth.uniform_device_residues((1, 2), ctx.q, ctx.n, 33, dev)
    b_attr = synth.uniform_device_residues((1, 2), ctx.q, ctx.n, 34, dev)
    rows_j = [0, 1, 2, 3]
    t = timed(lambda: ctx.join_sum(x, b_key, b_attr, rows_j), 1)
    out["join"] = {"rows": rows, "reference_rows": len(rows_j), "ms": t * 1e3,
                   "ms_per_reference_row": t * 1e3 / len(rows_j),
                   "fact_records_per_s_per_reference_row": rows * len(rows_j) / t}
    log(f"JOIN ({len(rows_j)} reference rows) {t * 1e3:.1f} ms")
    return out


def summarize_profiles(prof_dir: str, out_dir: str) -> None:
    """Turn rocprofv3 output (kernel trace stats; FETCH_SIZE and WRITE_SIZE
    counter passes that include a device copy of known size) into the short
    summaries kept under profiles/.  Counter readings are scaled by the
    ratio of the copy's known bytes to what the same counter reads for it."""
    import csv
    import collections
    os.makedirs(out_dir, exist_ok=True)
    stats = list(csv.DictReader(open(os.path.join(prof_dir, "trace", "eq_kernel_stats.csv"))))
    lines = ["| kernel | calls | mean us | total ms | % |", "|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    mib = 256
    traffic = {}
    factors = {}
    per_kind = {}
    for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        rows = list(csv.DictReader(open(os.path.join(prof_dir, sub, "eq_counter_collection.csv"))))
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
                and int(r["Grid_Size"]) >= 131072]
        factor = (mib * 1024) / max(copy) if copy else 1.0
        factors[counter] = factor
        agg = collections.defaultdict(list)
        for r in rows:
            agg[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
        for (name, grid), v in agg.items():
            per_kind.setdefault((name, grid), {})[counter] = sum(v) / len(v) * 1024 * factor
    tl = ["| kernel | grid | fetch MB/launch | write MB/launch |", "|---|---|---|---|"]
    for (name, grid), d in sorted(per_kind.items(), key=lambda kv: -sum(kv[1].values())):
        if sum(d.values()) < 1e8:
            continue
        tl.append(f"| {name[:70]} | {grid} | {d.get('FETCH_SIZE', 0) / 1e6:.1f} | "
                  f"{d.get('WRITE_SIZE', 0) / 1e6:.1f} |")
    # the digit transform: the forward NTT in its digit modes (digits of one,
    # two or three primes), by coefficient parity or full-limb
    import re
    for (name, grid), d in per_kind.items():
        if re.search(r"k_ntt_fwd_par<[156],|k_ntt_fwd_half<[156]>|k_ntt_fwd<\d+, [156]>", name):
            traffic["ntt_digit"] = d.get("FETCH_SIZE", 0) + d.get("WRITE_SIZE", 0)
        if re.search(r"k_scale<", name):
            traffic["scale"] = d.get("FETCH_SIZE", 0) + d.get("WRITE_SIZE", 0)
    with open(os.path.join(out_dir, "traffic.json"), "w") as fh:
        json.dump({"kernel_hash": kernel_hash(), "bytes_per_launch": traffic,
                   "calibration": {"copy_mib": mib, "factors": factors}}, fh, indent=1)
    cmd_trace = (f"rocprofv3 --kernel-trace --stats -d {prof_dir}/trace -o eq --output-format csv "
                 "-- python3 bench.py --steps 3 --warmup 1 --skip-batched --skip-cpu --skip-next "
                 "--skip-latency --skip-probes --skip-other --streams 1")
    cmd_pmc = (f"rocprofv3 --pmc {{C}} -d {prof_dir}/{{d}} -o eq --output-format csv -- python3 "
               "bench.py --steps 1 --warmup 0 --skip-batched --skip-cpu --skip-next --skip-latency "
               "--skip-probes --skip-other --streams 1 --calibrate-copy-mib 256")
    with open(os.path.join(out_dir, "eq_mask_2p20_rows_kernels.md"), "w") as fh:
        fh.write("# EQ mask, 2^20 rows (32 ciphertexts, N=32768), per-kernel time\n\n")
        fh.write(f"Library hash: {kernel_hash()}\n\nCommand (from the repo root, "
                 f"TMPDIR=/tmp):\n\n    {cmd_trace}\n\n")
        fh.write("\n".join(lines) + "\n")
    with open(os.path.join(out_dir, "eq_mask_2p20_rows_hbm_traffic.md"), "w") as fh:
        fh.write("# EQ mask, 2^20 rows: HBM bytes per launch (FETCH_SIZE, WRITE_SIZE)\n\n")
        fh.write(f"Library hash: {kernel_hash()}\n\nCommands, one counter per pass:\n\n")
        fh.write("    " + cmd_pmc.format(C="FETCH_SIZE", d="fetch") + "\n")
        fh.write("    " + cmd_pmc.format(C="WRITE_SIZE", d="write") + "\n\n")
        fh.write(f"Calibration: a {mib} MiB device copy reads {mib} MiB and writes {mib} MiB; "
                 f"scale factors applied: {json.dumps(factors)}.\n\n")
        fh.write("\n".join(tl) + "\n")


def main() -> int:
    if len(sys.argv) >= 2 and sys.argv[1] == "--summarize-profiles":
        summarize_profiles(sys.argv[2], os.path.join(ROOT, "profiles"))
        return 0
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-ct", type=int, default=32, help="ciphertexts per column (2^20 rows)")
    ap.add_argument("--batched-instances", type=int, default=512)
    ap.add_argument("--batched-reps", type=int, default=1)
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time one 32,768-slot ciphertext's whole oracle EQ on one core "
                         "(about 1.5 minutes)")
    ap.add_argument("--skip-probes", action="store_true")
    ap.add_argument("--ks-fused", type=int, default=-1,
                    help="key-switch product fused with the digit transforms (1) or not (0); "
                         "default: the context's tuning")
    ap.add_argument("--skip-latency", action="store_true",
                    help="skip the one-ciphertext latency runs (profiling: keeps every "
                         "launch at the column's size)")
    ap.add_argument("--skip-next", action="store_true",
                    help="skip IN / SELECT / SUM over the same column")
    ap.add_argument("--next-reps", type=int, default=2)
    ap.add_argument("--alpha", type=int, default=3, choices=(1, 2, 3),
                    help="data primes per key-switching digit: 3 (15 data primes, three special "
                         "primes; the default: the fastest whose noise budget covers every "
                         "operator), 2 (16 data primes, two special primes) or 1 (17 data "
                         "primes and one special prime)")
    ap.add_argument("--streams", type=int, default=0, choices=(0, 1, 2),
                    help="EQ calls on one stream (1) or the column's halves on two (2); "
                         "default: the context's tuning (two).  The rocprofv3 runs use 1, so "
                         "that every launch covers the whole column alone on the GPU")
    ap.add_argument("--skip-other", action="store_true",
                    help="skip timing the other key-switching decompositions")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(ciphertexts shard with no communication; see the design notes)", file=sys.stderr)
        return 2

    cp = None
    if not args.skip_cpu:
        cp = cpu_phase(args.cpu_full, args.alpha)

    import torch
    import synth
    from paper_2602_24271_amd import Context

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 2
    dev = torch.device("cuda", 0)
    if args.calibrate_copy_mib:
        a = torch.empty(args.calibrate_copy_mib << 17, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    n_ct = args.n_ct
    ctx, x, y, out = eq_setup(args.alpha, n_ct, args.ks_fused, dev, args.streams)
    ms, prof, margin, ms_one = eq_steps(ctx, x, y, out, args.steps, args.warmup)
    records = n_ct * ctx.n
    value = records / (ms / 1e3)
    log(f"{ms:.2f} ms/step, {value:.4g} records/s")
    roof, roof_ntt = roofline_dominant(prof, ctx)
    rates = derived_rates(ctx, prof, args.steps, n_ct, ms)
    roof_ks = roofline_ks(ctx, prof, n_ct, ctx.tuning()["ks_chunk"])
    # the other key-switching decompositions on the same column, same steps
    other = None
    if not args.skip_other:
        other = []
        for oa in (1, 2, 3):
            if oa == args.alpha:
                continue
            c2, x2, y2, o2 = eq_setup(oa, n_ct, -1, dev, args.streams)
            ms2, prof2, _, ms2_one = eq_steps(c2, x2, y2, o2, args.steps, args.warmup)
            other.append({"special_primes": oa, "data_primes": c2.L, "key_switch_digits": c2.dnum,
                          "depth_budget": c2.depth_budget,
                          "ms_per_step": ms2, "records_per_s": records / (ms2 / 1e3),
                          "ms_per_step_one_stream": ms2_one,
                          "roofline": roofline_dominant(prof2, c2)[0],
                          "roofline_ks_mac": roofline_ks(c2, prof2, n_ct, c2.tuning()["ks_chunk"]),
                          "kernels": {k: {"launches": v["launches"] // args.steps,
                                          "ms_per_step": v["ms"] / args.steps}
                                      for k, v in prof2.items()}})
            log(f"alpha={oa}: {ms2:.2f} ms/step, {records / (ms2 / 1e3):.4g} records/s")
            c2.close()
            del c2, x2, y2, o2
            torch.cuda.empty_cache()
    # one ciphertext (32,768 rows, the paper's per-query workload): latency
    lat_ms = None
    if not args.skip_latency:
        lat_ms = timed(lambda: ctx.eq_mask(x[:1], y[:1], out[:1]), 5) * 1e3
        log(f"one-ciphertext latency {lat_ms:.2f} ms")
    kernels = {k: {"launches": v["launches"] // args.steps, "ms_per_step": v["ms"] / args.steps}
               for k, v in prof.items()}

    nxt = None
    if not args.skip_next:
        nxt = next_rows(ctx, x, out, args.next_reps)
    bat = bat_fwd = None
    if not args.skip_batched:
        bat = batched(ctx, args.batched_instances, args.batched_reps)
        # 128 instances, rows log-uniform in [2^16, 2^20] (2..32 ciphertexts)
        bat_fwd = batched(ctx, 128, args.batched_reps, seed=3, lo_rows=1 << 16)
    cpu = check = None
    if cp is not None:
        cpu = cpu_baseline(cp)
        log(f"cpu baseline {cpu['value']:.1f} records/s on {cpu['cores']} cores")
        check = batched_check(cp, bat["wave_ct"] if bat else 4, args.alpha)
    prb = None if args.skip_probes else probes(ctx)

    line = {
        "metric": "hot-kernel elements/s + % roofline at 1 GPU; batched and adjoint vs plain",
        "value": value,
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_one_stream": ms_one,
        "schedule": {"timed": ("the column's two halves on two streams" if ms_one is not None
                               else "one stream"),
                     "kernels_and_roofline": "one stream: every launch timed alone on the GPU, "
                                             "covering the whole column"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"EQ mask (16 squarings + relinearization) over a column of "
                               f"{records} rows = {n_ct} BFV ciphertexts, N=32768, "
                               f"log2(QP)<=881 ({ctx.L}+{ctx.alpha} primes, key-switching "
                               f"digits of {ctx.alpha} prime{'s' if ctx.alpha > 1 else ''}), "
                               f"p=65537",
                   "rows": records, "ciphertexts": n_ct, "ring_degree": ctx.n,
                   "data_primes": ctx.L, "special_primes": ctx.alpha,
                   "key_switch_digits": ctx.dnum, "plaintext_modulus": ctx.t},
        "roofline": roof,
        "roofline_ntt_digit": roof_ntt if roof_ntt is not roof else None,
        "roofline_ks_mac": roof_ks,
        "other_key_switching": other,
        "cpu_baseline": cpu,
        "rates": rates,
        "latency_1ct_ms": lat_ms,
        "kernels": kernels,
        "batched": bat,
        "batched_128": bat_fwd,
        "batched_check": check,
        "probes": prb,
        "next_rows": nxt,
        "adjoint": None,
        "adjoint_note": "no adjoint: the mask is discrete (Z_t plaintexts, R_Q ciphertexts)",
        "margin_events": margin,
        "paper_context": {"records_per_s": PAPER_RECORDS_PER_S,
                          "hardware": "1 thread of a 16-core Intel Raptor Lake, Microsoft SEAL",
                          "source": "Table tab:primitive-times, Equality row (0.09 ms per record)"},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
