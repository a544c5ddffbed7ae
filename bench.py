#!/usr/bin/env python3
"""Throughput of the muffin-tin H+S build on one MI355X.

One step = one hsbuild_forward call (matching coefficients, per-atom T
products and the fused Hermitian H/S contraction) over the full-size
synthetic cell: 4 atom types x 32 atoms, l_max = 10 (N_L = 121), N_G = 12000,
complex128.  Inputs are resident in HBM before the timed region.  The value
is FP64-equivalent TFLOP/s with the algorithmic flop count
F = 16 k_c N_G (N_G + 1) + 32 N_atoms N_L^2 N_G  (k_c = N_atoms N_L).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

FP64_MFMA_PEAK_TFLOPS = 78.6
METRIC = "H+S build FP64-equiv TFLOP/s, % FP64 MFMA peak; split/FP64 speedup @1e-10"


def log(msg: str) -> None:
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def host_cpu() -> dict:
    """CPU model and physical core count of the host (from /proc/cpuinfo)."""
    model, cores = None, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name" and model is None:
                    model = val
                elif key == "physical id":
                    phys = val
                elif key == "core id":
                    core = val
                elif not key and phys is not None and core is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None and core is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return {"cpu_model": model, "physical_cores": len(cores) or None, "logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_baseline(index: int, n_g: int, split_forms=()) -> dict:
    """The oracle as it stands, on a bounded sample of the same workload: the
    same cell at a reduced basis size.  With split_forms ((name, precision,
    slices) triples), the oracle's H and S of the same cell at N_G = 3000 also
    serve as the reference for each split form's error, computed on the GPU at
    that size (the oracle stays on the host)."""
    from threadpoolctl import threadpool_info

    from flapw_cells import make_case
    from oracle import hs_oracle as o
    case = make_case(index, n_g=n_g)
    t0 = time.perf_counter()
    o.hs(case)
    dt = time.perf_counter() - t0
    flops = o.flops_forward(case["n_atoms"], case["n_l"], n_g)
    threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
    out = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
           "threads": int(threads), **host_cpu(),
           "sample": "oracle H+S (numpy complex128 over OpenBLAS, %d threads) on the same cell at N_G=%d "
                     "(F=%.3g TFLOP, %.1f s)" % (threads, n_g, flops / 1e12, dt)}
    if split_forms:
        import numpy as np
        import torch

        from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
        c3 = make_case(index, n_g=3000)
        Hr, Sr = o.hs(c3)
        g, tau, T = case_tensors(c3)
        errs = {}
        for name, precision, slices in split_forms:
            bs = HSBuilder.from_case(c3, precision=precision, n_slices=slices)
            H, S = bs.forward(c3["k_frac"], g, tau, T)
            H, S = H.cpu().numpy(), S.cpu().numpy()
            bs.close()
            full = lambda M: np.triu(M) + np.triu(M, 1).conj().T
            eh = float(np.linalg.norm(full(H) - Hr) / np.linalg.norm(Hr))
            es = float(np.linalg.norm(full(S) - Sr) / np.linalg.norm(Sr))
            errs["%s_x%d" % (name, slices)] = {"H": eh, "S": es, "meets_1e-10": bool(max(eh, es) <= 1e-10)}
            log("split %s x%d vs oracle at N_G=3000: H %.2e S %.2e" % (name, slices, eh, es))
        del g, tau, T
        torch.cuda.empty_cache()
        out["split_vs_oracle_ng3000"] = errs
    return out


def split_leg(args, case, b64, g, tau, T, H, S, ws, ms_fp64, flops) -> dict:
    """The split-precision forwards on the same workload (the residue form on the
    int8, BF16 and FP16 matrix cores, then int8, BF16 and FP16 slices): time per
    step, speedup over the FP64 path timed next to them and the relative Frobenius
    error against it.  The fastest form that meets the 1e-10 bar is the headline
    split figure."""
    import torch

    from paper_1712_07206_amd import (HSB_SPLIT_BF16, HSB_SPLIT_CRT, HSB_SPLIT_CRT_BF16, HSB_SPLIT_CRT_FP16,
                                      HSB_SPLIT_FP16, HSB_SPLIT_INT8)
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, hermitian_full
    n = case["n_g"]
    # the FP64 path re-timed next to the split ones, so all run at the same clock and temperature
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(2):
        code = b64.forward_raw(case["k_frac"], n, g, tau, T, H, S, ws, ws.numel())
        if code != N.HSB_OK:
            raise N.HSBuildError(code, N.last_error(b64._h))
    e1.record()
    torch.cuda.synchronize()
    ms_fp64_adj = e0.elapsed_time(e1) / 2
    H64, S64 = hermitian_full(H), hermitian_full(S)
    b64.close()
    del ws
    torch.cuda.empty_cache()

    def one(name, precision, slices, bits, peak, unit, kernel):
        bs = HSBuilder.from_case(case, precision=precision, n_slices=slices)
        wsb = bs.workspace_bytes(N.HSB_MODE_FORWARD, [n])
        wss = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        log("split %s x%d: workspace %.2f GB" % (name, slices, wsb / 1e9))

        def step():
            code = bs.forward_raw(case["k_frac"], n, g, tau, T, H, S, wss, wsb)
            if code != N.HSB_OK:
                raise N.HSBuildError(code, N.last_error(bs._h))

        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        bs.set_timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        stage_ms, _ = bs.stage_times()
        eh = (torch.linalg.norm(hermitian_full(H) - H64) / torch.linalg.norm(H64)).item()
        es = (torch.linalg.norm(hermitian_full(S) - S64) / torch.linalg.norm(S64)).item()
        if precision in (HSB_SPLIT_CRT, HSB_SPLIT_CRT_BF16, HSB_SPLIT_CRT_FP16):
            # residue-MFMA work of the two contraction launches (S and H): every 256 x 256 block of the
            # upper triangle, the stacked rows padded to 64, per modulus two int8 products (P and Q,
            # one workgroup each) x 2 operations
            nbs = -(-n // 256)
            k64 = -(-2 * case["n_atoms"] * case["n_l"] // 64) * 64
            mfma_ops = 2.0 * nbs * (nbs + 1) * 256 * 128 * k64 * slices * 2 * 2
        else:
            # slice-MFMA work executed by the two contraction launches (S and H): every 128 x 64 tile
            # of the upper triangle, the stacked rows padded to 32, S(S+1)/2 slice pairs x 4 real
            # products x 2 operations
            nbr = -(-n // 128)
            k_pad2 = -(-2 * case["n_atoms"] * case["n_l"] // 32) * 32
            pairs = slices * (slices + 1) // 2
            mfma_ops = 2.0 * nbr * (nbr + 1) * 128 * 64 * k_pad2 * pairs * 8
        rate = mfma_ops / (stage_ms[2] * 1e-3) / 1e12
        options = {"waves": bs.get_option(N.HSB_OPT_HS_WAVES), "tile_group": bs.get_option(N.HSB_OPT_TILE_GROUP)}
        log("split %s x%d: %.3f ms/step (contraction stage %.3f ms); FP64 path next to it %.3f ms: speedup %.3f; "
            "rel err vs FP64 H %.2e S %.2e" % (name, slices, ms, stage_ms[2], ms_fp64_adj, ms_fp64_adj / ms, eh, es))
        del wss
        bs.close()
        torch.cuda.empty_cache()
        return {"precision": name, "slices": slices, "slice_bits": bits, "kernel": kernel, "options": options,
                "ms_per_step": round(ms, 4),
                "fp64_equiv_tflops": round(flops / (ms * 1e-3) / 1e12, 4), "speedup": round(ms_fp64_adj / ms, 4),
                "fp64_ms_adjacent": round(ms_fp64_adj, 4), "speedup_vs_headline_fp64": round(ms_fp64 / ms, 4),
                "stages_ms": {"coefficients": round(stage_ms[0], 4),
                              "t_products_and_split_operands": round(stage_ms[1], 4),
                              "split_contraction": round(stage_ms[2], 4), "recombination": round(stage_ms[3], 4)},
                "rel_err_vs_fp64": {"H": eh, "S": es}, "meets_1e-10": bool(eh <= 1e-10 and es <= 1e-10),
                "slice_mfma": {"executed_ops": mfma_ops, "achieved": round(rate, 2), "peak": peak, "unit": unit,
                               "frac": round(rate / peak, 4)}}

    forms = []
    if args.crt_moduli > 0:  # "slices" of the residue form: its moduli; "slice_bits": bits per residue byte
        forms.append(one("crt", HSB_SPLIT_CRT, args.crt_moduli, 8, 5000.0, "TOP/s", "k_hs_crt"))
    if args.crt16_moduli > 0:  # the residues as bfloat16 / half integers on the 16-bit matrix cores
        forms.append(one("crt_bf16", HSB_SPLIT_CRT_BF16, args.crt16_moduli, 8, 2500.0, "TFLOP/s", "k_hs_crt"))
        forms.append(one("crt_fp16", HSB_SPLIT_CRT_FP16, args.crt16_moduli, 8, 2500.0, "TFLOP/s", "k_hs_crt"))
    if args.int8_slices > 0:
        forms.append(one("int8", HSB_SPLIT_INT8, args.int8_slices, 7, 5000.0, "TOP/s", "k_hs_split8"))
    if args.split_slices > 0:
        forms.append(one("bf16", HSB_SPLIT_BF16, args.split_slices, 8, 2500.0, "TFLOP/s", "k_hs_split2"))
    if args.fp16_slices > 0:
        forms.append(one("fp16", HSB_SPLIT_FP16, args.fp16_slices, 8, 2500.0, "TFLOP/s", "k_hs_split"))
    del H64, S64
    torch.cuda.empty_cache()
    # headline: the fastest form that meets the 1e-10 bar
    ok = [f for f in forms if f["meets_1e-10"]]
    best = min(ok, key=lambda f: f["ms_per_step"]) if ok else forms[0]
    out = dict(best)
    out["other_forms"] = [f for f in forms if f is not best]
    return out


def factored_flops(case, mac_flops=8.0) -> tuple:
    """Algorithmic flops of the type-factored forward: per upper-triangle entry and
    type, N_t + 4 N_L complex multiply-adds (phases, H and S slots; mac_flops each:
    8 in the conventional count, 6 as the 3M form executes them) and two complex
    products folded in; plus the per-type T products.  Returns (contraction, total)."""
    n, n_l = case["n_g"], case["n_l"]
    counts = [int((case["atom_type"] == t).sum()) for t in range(case["n_types"])]
    per_entry = sum(mac_flops * (nt + 4 * n_l) + 16.0 for nt in counts if nt > 0)
    contraction = per_entry * n * (n + 1) / 2.0
    return contraction, contraction + 32.0 * sum(1 for nt in counts if nt > 0) * n_l * n_l * n


def factored_leg(args, case, g, tau, T, H, S, ms_fp64) -> dict:
    """The type-factored forward (hsbuild_forward_factored) on the same workload:
    time to solution, speedup over the stacked FP64 path and the relative
    Frobenius error against its H and S (upper triangles)."""
    import torch

    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder
    n = case["n_g"]
    bf = HSBuilder.from_case(case)
    wsb = bf.workspace_bytes(N.HSB_MODE_FACTORED, [n])
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    H2 = torch.empty_like(H)
    S2 = torch.empty_like(S)
    log("factored path: workspace %.2f GB" % (wsb / 1e9))
    kf = case["k_frac"]

    for _ in range(max(1, args.warmup)):
        bf.forward_factored(kf, g, tau, T, H2, S2, ws=ws)
    torch.cuda.synchronize()
    bf.set_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(args.steps, 10)
    e0.record()
    for _ in range(reps):
        bf.forward_factored(kf, g, tau, T, H2, S2, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    stage_ms, _ = bf.stage_times()
    bf.set_timing(False)
    Hu, Su = torch.triu(H), torch.triu(S)
    eh = (torch.linalg.norm(torch.triu(H2) - Hu) / torch.linalg.norm(Hu)).item()
    es = (torch.linalg.norm(torch.triu(S2) - Su) / torch.linalg.norm(Su)).item()
    del Hu, Su, H2, S2, ws
    bf.close()
    torch.cuda.empty_cache()
    fc, ft = factored_flops(case)
    fx, _ = factored_flops(case, 6.0)  # as executed (3M form)
    kt = fc / (stage_ms[2] * 1e-3) / 1e12
    kx = fx / (stage_ms[2] * 1e-3) / 1e12
    log("factored: %.3f ms/step (contraction %.3f ms, %.2f TFLOP/s on its own %.4g TFLOP), %.1fx faster than the "
        "stacked FP64 path, rel err vs it H %.2e S %.2e" % (ms, stage_ms[2], kt, fc / 1e12, ms_fp64 / ms, eh, es))
    return {"ms_per_step": round(ms, 4), "steps": reps, "speedup_vs_fp64": round(ms_fp64 / ms, 3),
            "own_flops_per_step": ft, "own_tflops": round(ft / (ms * 1e-3) / 1e12, 4),
            "stages_ms": {"coefficients": round(stage_ms[0], 4), "t_products": round(stage_ms[1], 4),
                          "fact_contraction": round(stage_ms[2], 4)},
            "roofline": {"kernel": "k_hs_fact", "bound": "mfma", "achieved": round(kx, 4),
                         "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(kx / FP64_MFMA_PEAK_TFLOPS, 4), "algorithmic_flops_per_launch": fx,
                         "complex_form": "3M", "fp64_equiv_tflops": round(kt, 4)},
            "rel_err_vs_fp64": {"H": eh, "S": es}}


def hsdla_leg(args, case, g, tau, T, H, S, ms_fp64) -> dict:
    """The paper's BLAS sequence on rocBLAS (hsbuild_forward_hsdla), Alg. 3 and
    Alg. 1, on the same workload: time per build, the fused path's speedup over
    each and the relative Frobenius error against the fused path's H and S."""
    import torch

    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder
    n, n_at, n_l = case["n_g"], case["n_atoms"], case["n_l"]
    k_c = n_at * n_l
    bb = HSBuilder.from_case(case)
    wsb = bb.workspace_bytes(N.HSB_MODE_HSDLA, [n])
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    H2 = torch.empty_like(H)
    S2 = torch.empty_like(S)
    log("rocBLAS HSDLA: workspace %.2f GB" % (wsb / 1e9))
    out = {}
    Hu, Su = torch.triu(H), torch.triu(S)
    for alg, flops in ((3, 20.0 * k_c * n * n + 24.0 * n_at * n_l * n_l * n),
                       (1, 24.0 * k_c * n * n + 24.0 * n_at * n_l * n_l * n)):
        bb.forward_hsdla(alg, case["k_frac"], g, tau, T, H2, S2, ws=ws)  # warm (rocBLAS loads its kernels)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(1, min(args.steps, 3))
        e0.record()
        for _ in range(reps):
            bb.forward_hsdla(alg, case["k_frac"], g, tau, T, H2, S2, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        eh = (torch.linalg.norm(torch.triu(H2) - Hu) / torch.linalg.norm(Hu)).item()
        es = (torch.linalg.norm(torch.triu(S2) - Su) / torch.linalg.norm(Su)).item()
        log("rocBLAS Alg. %d: %.3f ms/build (%.2f TFLOP/s on its own %.4g TFLOP); fused FP64 path %.2fx faster; "
            "rel err vs fused H %.2e S %.2e" % (alg, ms, flops / (ms * 1e-3) / 1e12, flops / 1e12, ms / ms_fp64, eh, es))
        out["alg%d" % alg] = {"ms_per_build": round(ms, 4), "reps": reps, "paper_flops": flops,
                              "tflops_on_paper_flops": round(flops / (ms * 1e-3) / 1e12, 4),
                              "fused_speedup": round(ms / ms_fp64, 4), "rel_err_vs_fused": {"H": eh, "S": es}}
    del Hu, Su, H2, S2, ws
    bb.close()
    torch.cuda.empty_cache()
    out["note"] = "rocBLAS zherk/zher2k/zherkx/zgemm/zhemm in the order of the paper's algorithms, same GPU and inputs"
    return out


def real_leg(args) -> dict:
    """The inversion-symmetric cell of the bench shape (4 types x 32 atoms as 16
    inversion pairs each, l_max 10, N_G 12000): hsbuild_forward (complex) and
    hsbuild_forward_real (real symmetric) on the same inputs; time of each and
    the difference of the real outputs from the complex ones' real parts."""
    import numpy as np
    import torch

    from flapw_cells import make_case
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(6)
    n, n_at, n_l = case["n_g"], case["n_atoms"], case["n_l"]
    n_rep = int((case["partner"] >= np.arange(n_at)).sum())
    flops_c = 16.0 * n_at * n_l * n * (n + 1) + 32.0 * n_at * n_l * n_l * n
    flops_r = 8.0 * n_rep * n_l * n * (n + 1) + 32.0 * n_rep * n_l * n_l * n
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    Hc = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    Sc = torch.empty_like(Hc)
    Hr = torch.empty((n, n), dtype=torch.float64, device="cuda")
    Sr = torch.empty_like(Hr)
    wsb = max(b.workspace_bytes(N.HSB_MODE_FORWARD, [n]), b.workspace_bytes(N.HSB_MODE_REAL, [n]))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    kf = case["k_frac"]
    reps = max(1, min(args.steps, 3))
    ms_c = timed(lambda: b.forward(kf, g, tau, T, Hc, Sc, ws=ws), reps)
    ms_r = timed(lambda: b.forward_real(kf, g, tau, case["partner"], T, Hr, Sr, ws=ws), reps)
    Hcu, Scu = torch.triu(Hc), torch.triu(Sc)
    imag = (torch.linalg.norm(Hcu.imag) / torch.linalg.norm(Hcu)).item()
    eh = (torch.linalg.norm(torch.triu(Hr) - Hcu.real) / torch.linalg.norm(Hcu.real)).item()
    es = (torch.linalg.norm(torch.triu(Sr) - Scu.real) / torch.linalg.norm(Scu.real)).item()
    Hr64, Sr64 = torch.triu(Hr), torch.triu(Sr)
    del Hc, Sc, Hcu, Scu, ws
    b.close()
    torch.cuda.empty_cache()
    # the split forms of the real path (int8 slices, residues), against the FP64 real path's outputs
    def real_split(name, precision, slices):
        bi = HSBuilder.from_case(case, precision=precision, n_slices=slices)
        wsi = bi.workspace(N.HSB_MODE_REAL, [n])
        ms_i = timed(lambda: bi.forward_real(kf, g, tau, case["partner"], T, Hr, Sr, ws=wsi), reps)
        ehi = (torch.linalg.norm(torch.triu(Hr) - Hr64) / torch.linalg.norm(Hr64)).item()
        esi = (torch.linalg.norm(torch.triu(Sr) - Sr64) / torch.linalg.norm(Sr64)).item()
        log("real-symmetric %s x%d: %.3f ms (%.2fx the FP64 real path); rel err vs it H %.2e S %.2e"
            % (name, slices, ms_i, ms_r / ms_i, ehi, esi))
        del wsi
        bi.close()
        return {"slices": slices, "ms": round(ms_i, 4), "speedup_vs_fp64_real": round(ms_r / ms_i, 4),
                "rel_err_vs_fp64_real": {"H": ehi, "S": esi}, "meets_1e-10": bool(ehi <= 1e-10 and esi <= 1e-10)}

    int8 = crt = None
    if args.int8_slices > 0:
        from paper_1712_07206_amd import HSB_SPLIT_INT8
        int8 = real_split("int8", HSB_SPLIT_INT8, args.int8_slices)
    if args.crt_moduli > 0:
        from paper_1712_07206_amd import HSB_SPLIT_CRT
        crt = real_split("crt", HSB_SPLIT_CRT, args.crt_moduli)
    del Hr, Sr, Hr64, Sr64
    torch.cuda.empty_cache()
    log("real-symmetric %s: complex path %.3f ms, real path %.3f ms (%.2fx), %.2f TFLOP/s on its own %.4g TFLOP; "
        "rel err vs complex H %.2e S %.2e, |Im H|/|H| %.1e" % (case["name"], ms_c, ms_r, ms_c / ms_r,
                                                            flops_r / (ms_r * 1e-3) / 1e12, flops_r / 1e12, eh, es,
                                                            imag))
    return {"workload": case["name"], "n_g": n, "representatives": n_rep, "ms_complex": round(ms_c, 4),
            "ms_real": round(ms_r, 4), "speedup": round(ms_c / ms_r, 4), "flops_real": flops_r,
            "flops_complex": flops_c, "real_tflops": round(flops_r / (ms_r * 1e-3) / 1e12, 4),
            "complex_imag_rel": imag, "rel_err_vs_complex": {"H": eh, "S": es}, "int8_split": int8,
            "crt_split": crt}


def small_leg(args) -> dict:
    """One k-point of the 16-atom l_max 8 cell at N_G = 3000 (k_c = 1296): the whole
    forward, its contraction against the FP64 MFMA roofline (executed 3M flops), in the
    library's default stream-K form (600 tiles: fewer than 4 per compute unit), with the
    stacked index in two segments, and in one pass."""
    import torch

    from flapw_cells import make_case
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(1)
    n, n_at, n_l = case["n_g"], case["n_atoms"], case["n_l"]
    k_c = n_at * n_l
    flops = 16.0 * k_c * n * (n + 1) + 32.0 * n_at * n_l * n_l * n
    flops_exec = 12.0 * k_c * n * (n + 1)
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    H = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    S = torch.empty_like(H)
    reps = max(10, 4 * args.steps)
    out = {"workload": case["name"], "n_g": n, "k_c": k_c, "flops_per_step": flops,
           "algorithmic_flops_per_launch": flops_exec}
    # auto: the stream-K contraction (equal shares of (tile, chunk) units per workgroup); 2: the
    # stacked index in two segments; 0: one pass
    for mode, key in ((1, "split_k_auto"), (2, "segments_2"), (0, "one_pass")):
        b.set_option(N.HSB_OPT_SPLIT_K, mode)
        wsb = b.workspace_bytes(N.HSB_MODE_FORWARD, [n])
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        for _ in range(3):
            code = b.forward_raw(case["k_frac"], n, g, tau, T, H, S, ws, wsb)
            if code != N.HSB_OK:
                raise N.HSBuildError(code, N.last_error(b._h))
        torch.cuda.synchronize()
        b.set_timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            code = b.forward_raw(case["k_frac"], n, g, tau, T, H, S, ws, wsb)
            if code != N.HSB_OK:
                raise N.HSBuildError(code, N.last_error(b._h))
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        st, _ = b.stage_times()
        b.set_timing(False)
        del ws
        achieved = flops_exec / (st[2] * 1e-3) / 1e12
        out[key] = {"ms_per_step": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 4),
                    "stages_ms": {"coefficients": round(st[0], 4), "t_products": round(st[1], 4),
                                  "hs_contraction": round(st[2], 4), "segment_sum": round(st[3], 4)},
                    "roofline": {"kernel": {1: "k_hs_fp64_stream", 2: "k_hs_fp64_sk", 0: "k_hs_fp64"}[mode],
                                 "bound": "mfma",
                                 "achieved": round(achieved, 4), "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4)}}
        log("N_G 3000 cell (%s): %.3f ms per forward, contraction %.3f ms = %.1f TFLOP/s executed (%.3f of peak), "
            "partial-tile sum %.3f ms" % (key, ms, st[2], achieved, achieved / FP64_MFMA_PEAK_TFLOPS, st[3]))
    b.close()
    torch.cuda.empty_cache()
    return out


def eigen_leg(args) -> dict:
    """The downstream generalized eigenproblem H c = lambda S c (rocSOLVER zhegvd
    through hsbuild_eigensolve) on the bench cell's H and S (built by the
    type-factored path), eigenvalues and eigenvectors."""
    import torch

    from flapw_cells import make_case
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(args.config, n_g=args.ng)
    n = case["n_g"]
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    H, S = b.forward_factored(case["k_frac"], g, tau, T)
    H0, S0 = H.clone(), S.clone()
    b.eigensolve(H, S, vectors=True)  # warm (rocSOLVER loads its kernels)
    H.copy_(H0)
    S.copy_(S0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    w, info = b.eigensolve(H, S, vectors=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    lo, hi = float(w[0]), float(w[-1])
    del H, S, H0, S0, w
    b.close()
    torch.cuda.empty_cache()
    log("eigensolve %s N_G=%d: %.1f ms with eigenvectors (rocSOLVER zhegvd), info %d, lambda in [%.4g, %.4g]"
        % (case["name"], n, ms, info, lo, hi))
    return {"workload": case["name"], "n_g": n, "ms_with_vectors": round(ms, 2), "info": info,
            "lambda_min": lo, "lambda_max": hi, "library": "rocSOLVER zhegvd"}


def batch_leg(args) -> dict:
    """The multi-k workload (64 k-points, N_G 2800-3400, T shared): one captured
    graph with a persistent contraction, against 64 sequential forward calls."""
    import torch

    from flapw_cells import make_batch_case
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder

    case = make_batch_case(3)
    n_k = len(case["g"])
    b = HSBuilder.from_case(case)
    tau = torch.as_tensor(case["tau"], device="cuda")
    T = torch.as_tensor(case["T"], device="cuda")
    gl = [torch.as_tensor(g, device="cuda") for g in case["g"]]
    ng = [int(x) for x in case["n_g"]]
    k_c = case["n_atoms"] * case["n_l"]
    flops = sum(16.0 * k_c * n * (n + 1) + 32.0 * case["n_atoms"] * case["n_l"] ** 2 * n for n in ng)
    from paper_1712_07206_amd import autotune
    tuned = autotune.tune_batch(b, case["k_frac"], gl, tau, T)
    log("batch autotuner: waves %d, tile group %d (%s)" % (tuned["waves"], tuned["tile_group"], ", ".join(
        "%s %.1f ms" % kv for kv in tuned["candidates_ms"].items())))
    H, S, off = b.batch(case["k_frac"], gl, tau, T)  # captures the graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps)
    e0.record()
    for _ in range(reps):
        b.batch(case["k_frac"], gl, tau, T, H, S)
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / reps
    # sequential: one forward per k on the same stream, outputs written in place, with the
    # library's default (stream-K on these small bases) and with the one-pass form
    outs = [(H[int(off[k]): int(off[k]) + ng[k] ** 2].view(ng[k], ng[k]),
             S[int(off[k]): int(off[k]) + ng[k] ** 2].view(ng[k], ng[k])) for k in range(n_k)]
    seq = {}
    for mode, key in ((1, "split_k_auto"), (0, "one_pass")):
        b.set_option(N.HSB_OPT_SPLIT_K, mode)
        wsb = max(b.workspace_bytes(N.HSB_MODE_FORWARD, [n]) for n in ng)  # the split's partials vary with n
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")

        def all_k():
            for k in range(n_k):
                code = b.forward_raw(case["k_frac"][k], ng[k], gl[k], tau, T, outs[k][0], outs[k][1], ws, wsb)
                if code != N.HSB_OK:
                    raise N.HSBuildError(code, N.last_error(b._h))

        all_k()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            all_k()
        e1.record()
        torch.cuda.synchronize()
        seq[key] = e0.elapsed_time(e1) / reps
        del ws
    ms_seq = seq["split_k_auto"]
    log("batch %d k-points: graph %.3f ms, sequential %.3f ms (one-pass %.3f ms), speedup %.3f (%.3f), %.2f TFLOP/s"
        % (n_k, ms_graph, ms_seq, seq["one_pass"], ms_seq / ms_graph, seq["one_pass"] / ms_graph,
           flops / (ms_graph * 1e-3) / 1e12))
    del H, S, outs
    b.close()
    torch.cuda.empty_cache()
    return {"workload": case["name"], "n_k": n_k, "n_g_min": min(ng), "n_g_max": max(ng),
            "ms_graph": round(ms_graph, 4), "ms_sequential": round(ms_seq, 4),
            "ms_sequential_one_pass": round(seq["one_pass"], 4),
            "speedup": round(ms_seq / ms_graph, 4), "speedup_vs_one_pass": round(seq["one_pass"] / ms_graph, 4),
            "fp64_equiv_tflops": round(flops / (ms_graph * 1e-3) / 1e12, 4),
            "autotuned": {"waves": tuned["waves"], "tile_group": tuned["tile_group"],
                          "candidates_ms": {k: round(v, 3) for k, v in tuned["candidates_ms"].items()}}}


def adjoint_leg(args) -> dict:
    """hsbuild_backward on the differentiation workload (64 atoms, l_max 10,
    N_G 6000; Hermitian W, V as dL/dH, dL/dS): time per call and FP64 rate for
    F_adj = 32 k_c N_G^2 + 64 N_atoms N_L^2 N_G."""
    import torch

    from flapw_cells import make_case
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors

    case = make_case(4)
    n, n_at, n_l = case["n_g"], case["n_atoms"], case["n_l"]
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    gH = torch.as_tensor(case["W"], device="cuda")
    gS = torch.as_tensor(case["V"], device="cuda")
    gT, gtau = b.backward(case["k_frac"], g, tau, T, gH, gS)  # warm, allocates the workspace
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps)
    e0.record()
    for _ in range(reps):
        b.backward(case["k_frac"], g, tau, T, gH, gS, gT, gtau)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 32.0 * n_at * n_l * n * n + 64.0 * n_at * n_l * n_l * n
    log("adjoint %s: %.3f ms per backward, %.2f TFLOP/s" % (case["name"], ms, flops / (ms * 1e-3) / 1e12))
    b.close()
    del gH, gS, gT, gtau
    torch.cuda.empty_cache()
    return {"workload": case["name"], "n_g": n, "ms_per_backward": round(ms, 4), "flops": flops,
            "fp64_equiv_tflops": round(flops / (ms * 1e-3) / 1e12, 4),
            "note": "conventional flop count; the products P_H, P_S run in the 3M form (6 flops per complex "
                    "multiply-add)"}


def coefficient_leg(case, ms_coef: float) -> dict:
    """The coefficient build (a1-a5, ending in the W write) as an HBM-bound
    stage: algorithmic bytes 2 k_c N_G x 16 (the coefficients written once)
    over the forward's coefficient stage time, against 8 TB/s and against a
    timed 2 GiB device-to-device copy (its read and its write both counted)."""
    import torch
    k_c = case["n_atoms"] * case["n_l"]
    alg = 2.0 * k_c * case["n_g"] * 16
    size = 2 << 30
    src = torch.empty(size, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None or ms < best else best
    del src, dst
    torch.cuda.empty_cache()
    copy_gbs = 2.0 * size / (best * 1e-3) / 1e9
    ach = alg / (ms_coef * 1e-3) / 1e9
    log("coefficient build: %.3f ms, %.0f GB/s (%.1f %% of 8 TB/s, %.1f %% of a %.0f GB/s copy)"
        % (ms_coef, ach, 100 * ach / 8000.0, 100 * ach / copy_gbs, copy_gbs))
    return {"stage": "a1-a5: tables, lambda and k_assemble (the W write)", "ms": round(ms_coef, 4),
            "algorithmic_bytes": alg, "achieved_gbs": round(ach, 1), "peak_gbs": 8000.0,
            "frac": round(ach / 8000.0, 4), "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(ach / copy_gbs, 4),
            "copy": "2 GiB device-to-device, read and write both counted"}


def device_leg() -> dict:
    """CU count, and the sustained matrix-core rates of the two instructions the
    contractions run on (FP64 16x16x4 and int8 32x32x32, the latter on constant
    and on changing random operands), measured by the library's probe; each rate
    divided by the per-CU rate per clock gives the clock the matrix cores hold
    under that load."""
    import torch

    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import mfma_probe
    props = torch.cuda.get_device_properties(0)
    cus = int(props.multi_processor_count)
    out = {"name": props.name, "arch": getattr(props, "gcnArchName", ""), "cus": cus}
    # per CU per clock: 4 SIMDs x (2048 FP64 operations per 64 cycles | 65536 int8 operations per 32 cycles)
    for key, kind, iters, per_clk, peak in (("fp64", N.HSB_PROBE_FP64, 50000, 128.0, 78.6),
                                            ("int8", N.HSB_PROBE_INT8, 100000, 8192.0, 5000.0),
                                            ("int8_random", N.HSB_PROBE_INT8_RANDOM, 100000, 8192.0, 5000.0)):
        blocks = 8 * cus
        ops, buf = mfma_probe(kind, blocks, 160)
        torch.cuda.synchronize()
        best = None
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ops, buf = mfma_probe(kind, blocks, iters, buf)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None or ms < best else best
        rate = ops / (best * 1e-3) / 1e12
        out[key + "_mfma_probe"] = {"achieved": round(rate, 2), "unit": "TFLOP/s" if key == "fp64" else "TOP/s",
                                    "peak": peak, "frac": round(rate / peak, 4), "ms": round(best, 3),
                                    "clock_ghz": round(rate * 1e12 / (cus * per_clk) / 1e9, 3)}
        log("%s MFMA probe: %.1f %s (%.1f %% of %.1f), %.3f GHz" % (key, rate, out[key + "_mfma_probe"]["unit"],
                                                                    100 * rate / peak, peak,
                                                                    out[key + "_mfma_probe"]["clock_ghz"]))
        del buf
    return out


def oracle_table() -> list:
    """The oracle on the host next to the GPU path at the same sizes: forward at
    cfg0, cfg1 (N_G 3000, also single-threaded) and cfg2 at N_G 3000, and the
    gradient at the differentiation cell at N_G 800."""
    import torch
    from threadpoolctl import threadpool_info, threadpool_limits

    from flapw_cells import make_case
    from oracle import hs_oracle as o
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])

    def gpu_ms(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    rows = []
    for idx, n_g, single in ((0, None, False), (1, 3000, False), (1, 3000, True), (2, 3000, False)):
        case = make_case(idx, n_g=n_g)
        n = case["n_g"]
        flops = o.flops_forward(case["n_atoms"], case["n_l"], n)
        t0 = time.perf_counter()
        if single:
            with threadpool_limits(limits=1, user_api="blas"):
                o.hs(case)
        else:
            o.hs(case)
        dt = time.perf_counter() - t0
        b = HSBuilder.from_case(case)
        g, tau, T = case_tensors(case)
        ms = gpu_ms(lambda: b.forward(case["k_frac"], g, tau, T))
        b.close()
        rows.append({"what": "forward", "workload": case["name"], "n_g": n, "oracle_threads": 1 if single else threads,
                     "oracle_s": round(dt, 4), "oracle_gflops": round(flops / dt / 1e9, 2), "gpu_ms": round(ms, 4),
                     "gpu_tflops": round(flops / (ms * 1e-3) / 1e12, 3), "ratio": round(dt * 1e3 / ms, 1)})
        log("oracle table: %s" % json.dumps(rows[-1]))
    case = make_case(4, n_g=800)
    n = case["n_g"]
    t0 = time.perf_counter()
    o.loss_gradients(case, case["W"], case["V"])
    dt = time.perf_counter() - t0
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    gH = torch.as_tensor(case["W"], device="cuda")
    gS = torch.as_tensor(case["V"], device="cuda")
    ms = gpu_ms(lambda: b.backward(case["k_frac"], g, tau, T, gH, gS))
    b.close()
    rows.append({"what": "gradient", "workload": case["name"], "n_g": n, "oracle_threads": threads,
                 "oracle_s": round(dt, 4), "gpu_ms": round(ms, 4), "ratio": round(dt * 1e3 / ms, 1),
                 "note": "the oracle's gradient takes the per-atom route (different from the GPU's adjoint)"})
    log("oracle table: %s" % json.dumps(rows[-1]))
    return rows


def recorded_traffic(workload: str, options: dict):
    """HBM bytes per launch of the contraction kernel from the committed
    rocprofv3 PMC record, only if the kernel source and its options are the
    ones profiled."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        rec = json.load(open(os.path.join(root, "profiles", "k_hs_fp64_traffic.json")))
        srcs = rec["source"] if isinstance(rec["source"], list) else [rec["source"]]
        src = b"".join(open(os.path.join(root, f), "rb").read() for f in srcs)
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("source_sha256_16") or rec.get("workload") != workload:
        return None
    if rec.get("options") != options:
        return None
    return rec["traffic_bytes"]


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, help="workload index (default: the full-size cell)")
    ap.add_argument("--ng", type=int, default=None, help="override the basis size")
    ap.add_argument("--cpu-ng", type=int, default=6600, help="basis size of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-table", action="store_true",
                    help="also time the oracle at cfg0, cfg1, cfg2 (N_G 3000) and the gradient, next to the GPU")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-k-point batch leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner before timing (default: the library's default options)")
    ap.add_argument("--waves", type=int, default=0, help="contraction waves per workgroup (4 or 8; skips tuning)")
    ap.add_argument("--tile-group", type=int, default=None, help="contraction tile order (skips tuning)")
    ap.add_argument("--no-factored", action="store_true", help="skip the type-factored leg")
    ap.add_argument("--no-hsdla", action="store_true", help="skip the rocBLAS HSDLA baseline leg")
    ap.add_argument("--no-real", action="store_true", help="skip the real-symmetric (inversion) leg")
    ap.add_argument("--no-small", action="store_true", help="skip the one-k-point N_G 3000 leg (16-atom cell)")
    ap.add_argument("--no-eigen", action="store_true", help="skip the generalized eigensolve leg")
    ap.add_argument("--no-device-probe", action="store_true", help="skip the matrix-core rate probe")
    ap.add_argument("--split-slices", type=int, default=5,
                    help="also time the BF16 split-precision path with this many slices (0: skip)")
    ap.add_argument("--int8-slices", type=int, default=6,
                    help="also time the int8 split-precision path with this many slices (0: skip)")
    ap.add_argument("--fp16-slices", type=int, default=5,
                    help="also time the FP16 split-precision path with this many slices (0: skip)")
    ap.add_argument("--crt-moduli", type=int, default=11,
                    help="also time the residue (CRT) split-precision path with this many moduli (0: skip)")
    ap.add_argument("--crt16-moduli", type=int, default=11,
                    help="also time the residue form on the BF16 and FP16 matrix cores with this many moduli "
                         "(0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the H/S tiles would be "
              "dealt over GPUs with no exchange; see the design notes). Run with --gpus 1.")
        return 2

    import numpy as np
    import torch

    from flapw_cells import make_case
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors

    if not torch.cuda.is_available():
        log("no HIP device")
        return 1
    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d MiB device-to-device" % args.copy_probe_mib)
        del src, dst
    case = make_case(args.config, n_g=args.ng)
    n, n_at, n_l = case["n_g"], case["n_atoms"], case["n_l"]
    k_c = n_at * n_l
    flops_hs = 16.0 * k_c * n * (n + 1)
    flops = flops_hs + 32.0 * n_at * n_l * n_l * n
    log("workload %s: N_G=%d atoms=%d N_L=%d k_c=%d F=%.4g TFLOP" % (case["name"], n, n_at, n_l, k_c, flops / 1e12))

    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    H = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    S = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    from paper_1712_07206_amd import _native as N
    ws_bytes = b.workspace_bytes(N.HSB_MODE_FORWARD, [n])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    log("workspace %.2f GB, outputs %.2f GB" % (ws_bytes / 1e9, 2 * H.numel() * 16 / 1e9))

    def step():
        code = b.forward_raw(case["k_frac"], n, g, tau, T, H, S, ws, ws_bytes)
        if code != N.HSB_OK:
            raise N.HSBuildError(code, N.last_error(b._h))

    tuned = None
    if args.waves or args.tile_group is not None:
        if args.waves:
            b.set_option(N.HSB_OPT_HS_WAVES, args.waves)
        if args.tile_group is not None:
            b.set_option(N.HSB_OPT_TILE_GROUP, args.tile_group)
    elif args.tune:
        from paper_1712_07206_amd import autotune
        del ws
        tuned = autotune.tune(b, case["k_frac"], g, tau, T, reps=1, path=None)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        log("autotuned contraction: waves %d, tile group %d (%s)"
            % (tuned["waves"], tuned["tile_group"], ", ".join("%s %.1f ms" % kv for kv in tuned["candidates_ms"].items())))
    options = {"waves": b.get_option(N.HSB_OPT_HS_WAVES), "tile_group": b.get_option(N.HSB_OPT_TILE_GROUP)}

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    b.set_timing(True)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    stage_ms, calls = b.stage_times()
    b.set_timing(False)
    ms_step = ms_total / args.steps
    log("timed %d steps: %.3f ms/step (wall %.3f s); stages ms: coef %.3f, tprod %.3f, hs %.3f over %d calls"
        % (args.steps, ms_step, wall, stage_ms[0], stage_ms[1], stage_ms[2], calls))
    tflops = flops / (ms_step * 1e-3) / 1e12
    # The 8-wave contraction forms each complex product from three real ones
    # (12 instead of 16 flops per stacked row and upper-triangle entry pair), the
    # 4-wave one from four: the roofline prices the kernel on the products it
    # has to execute, the headline on the conventional count.
    flops_hs_exec = (12.0 if options["waves"] == 8 else 16.0) * k_c * n * (n + 1)
    hs_tflops = flops_hs_exec / (stage_ms[2] * 1e-3) / 1e12
    hs_equiv = flops_hs / (stage_ms[2] * 1e-3) / 1e12

    result = {
        "metric": METRIC,
        "value": round(tflops, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded cell, positions, radial values and Hermitian T blocks shaped like the "
                "paper's workloads (no FLEUR inputs)",
        "config": {"workload": case["name"], "n_atoms": n_at, "n_types": case["n_types"], "l_max": case["l_max"],
                   "n_l": n_l, "n_g": n, "k_c": k_c, "precision": "fp64", "flops_per_step": flops},
        "pct_fp64_mfma_peak": round(100.0 * tflops / FP64_MFMA_PEAK_TFLOPS, 2),
        "pct_note": "FP64-equivalent rate (conventional 8-flop complex multiply-add count) over the FP64 MFMA "
                    "peak; the 3-product complex form lets it pass 100%",
        "contraction_options": options,
        "stages_ms": {"coefficients": round(stage_ms[0], 4), "t_products": round(stage_ms[1], 4),
                      "hs_contraction": round(stage_ms[2], 4), "segment_sum": round(stage_ms[3], 4)},
        "roofline": {"kernel": "k_hs_fp64", "bound": "mfma", "achieved": round(hs_tflops, 4),
                     "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(hs_tflops / FP64_MFMA_PEAK_TFLOPS, 4),
                     "traffic": recorded_traffic(case["name"], options),
                     "algorithmic_flops_per_launch": flops_hs_exec,
                     "complex_form": "3M" if options["waves"] == 8 else "4M",
                     "fp64_equiv_tflops": round(hs_equiv, 4)},
        "split_speedup": None,
        "paper_context": {
            "note": "the paper's figures on its own hardware and inputs: context, not a target",
            "abstract": "over 70% of peak on CPU+coprocessor nodes; 5x over CPU-only on a JURECA node",
            "sec6_rwth_gpu": "about 2 of 3 TFLOP/s (66%); TiO2 at K_max 4.0 about 2.5 TFLOP/s (83%)",
            "sec6_jureca_gpu": "4 GK210 + 2 Haswell, 6.7 TFLOP/s peak: up to 3.2 TFLOP/s AuAg (47%), 4.3 TFLOP/s "
                               "TiO2 (61%), whole H/S build",
        },
    }
    result["coefficient_build"] = coefficient_leg(case, stage_ms[0])
    if not args.no_factored:
        result["factored"] = factored_leg(args, case, g, tau, T, H, S, ms_step)
    if not args.no_hsdla:
        result["hsdla_rocblas"] = hsdla_leg(args, case, g, tau, T, H, S, ms_step)
    if args.split_slices > 0 or args.int8_slices > 0 or args.fp16_slices > 0 or args.crt_moduli > 0 or \
            args.crt16_moduli > 0:
        result["split"] = split_leg(args, case, b, g, tau, T, H, S, ws, ms_step, flops)
        if result["split"]["meets_1e-10"]:
            result["split_speedup"] = result["split"]["speedup"]
    del H, S, ws
    torch.cuda.empty_cache()
    if not args.no_small:
        result["cfg1"] = small_leg(args)
    if not args.no_real:
        result["real_symmetric"] = real_leg(args)
    if not args.no_adjoint:
        result["adjoint"] = adjoint_leg(args)
    if not args.no_eigen:
        result["eigensolve"] = eigen_leg(args)
    if not args.no_batch:
        result["batch"] = batch_leg(args)
        result["batch_speedup"] = result["batch"]["speedup"]
    if not args.no_device_probe:
        result["device"] = device_leg()
        # each kernel's rate against what the matrix cores sustain on this device (the probe)
        dev = result["device"]
        result["roofline"]["probe_frac"] = round(result["roofline"]["achieved"] / dev["fp64_mfma_probe"]["achieved"], 4)
        for form in ([result["split"]] + result["split"]["other_forms"]) if result.get("split") else []:
            if form["precision"] in ("int8", "crt"):
                sm = form["slice_mfma"]
                sm["probe_frac"] = round(sm["achieved"] / dev["int8_mfma_probe"]["achieved"], 4)
                # against the rate the int8 matrix cores hold on random operands (power-bound)
                sm["random_probe_frac"] = round(sm["achieved"] / dev["int8_random_mfma_probe"]["achieved"], 4)
    if not args.no_cpu_baseline:
        log("timing the oracle sample on the host (N_G=%d)" % args.cpu_ng)
        from paper_1712_07206_amd import HSB_SPLIT_BF16, HSB_SPLIT_CRT, HSB_SPLIT_FP16, HSB_SPLIT_INT8
        forms = [("crt", HSB_SPLIT_CRT, args.crt_moduli), ("int8", HSB_SPLIT_INT8, args.int8_slices),
                 ("bf16", HSB_SPLIT_BF16, args.split_slices), ("fp16", HSB_SPLIT_FP16, args.fp16_slices)]
        result["cpu_baseline"] = cpu_baseline(args.config, args.cpu_ng, [f for f in forms if f[2] > 0])
        log("oracle: %.4f TFLOP/s on %d threads" % (result["cpu_baseline"]["value"], result["cpu_baseline"]["cores"]))
    else:
        result["cpu_baseline"] = None
    if args.oracle_table:
        result["oracle_table"] = oracle_table()
    print(json.dumps(result))
    sys.stdout.flush()
    return 0


if __name__ == "__main__":
    sys.exit(main())
