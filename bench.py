"""Benchmark: FP64 CRS spMVM on the permuted 3D stencil with random extras
(N = 21,952,000 rows, 170M nonzeros), one MI355X -- the largest workload, on
which the headline is quoted.

One step = one C = A*B product through spmv_apply with the plan's variant
(autotuned), inputs resident in HBM. Prints ONE JSON line (rank 0) with
GFlop/s, the roofline of the product kernel (HBM-bound: the bytes the
kernel must read / kernel time, against 8 TB/s, with the HBM bytes the
counters measured), and the CPU oracle timed on the host as a baseline next
to the paper's node scheme on all host cores. Extra measurements (the
Hamiltonian-like workload with the best kernel on the caller's CRS arrays and
the chunked copy, FP32 storage, multi-RHS, the uneven batch, RCM, solvers, a
triad) go into "extra".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CRS spMVM GFlop/s and effective HBM GB/s (% roofline) at 1 MI355X, FP64 vs mixed"
HBM_PEAK = 8000.0  # GB/s, MI355X nominal
KERNEL_NAMES = {"V4_lds_block": "k_lds_block<double,double>",
                "V4_lds_block_staged": "k_lds_block_staged<double,double>",
                "V4_lds_block_windows": "k_win_rows<double,double,true>",
                "V6_sell64": "k_sell_pairs"}
# the paper's own CPU figures (Sect. 2, one Xeon X5550 socket, HMeP matrix):
# context only, another machine and another matrix
PAPER_CPU = {"hardware": "Intel Xeon X5550 (Nehalem EP, 4 cores, 2.66 GHz), one socket",
             "matrix": "HMeP Holstein-Hubbard, N=6.2e6, N_nzr~15",
             "spmv_gflops": 2.25, "spmv_gbs": 18.1, "stream_triad_gbs": 21.2,
             "model_bound_gflops_at_18.1GBs": 2.66}
SELL = 0  # plan flag requesting the V6 chunked copy; set in main()
# multi-RHS products kept for the accuracy report: per (precision, k) the GPU's
# C on a seeded row sample, with the sample's rows of A (see spmm_samples)
SPMM_SAMPLES: list = []
SPMM_SAMPLE_ROWS = 4096


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# sources that define each variant's product kernel (a stored counter record
# is valid only while these files are unchanged)
KERNEL_SOURCES = {"V6_sell64": ("sell.hip", "device.hpp", "common.hpp"),
                  # the staged form's B ranges are chosen at create (analysis.hip)
                  "V4_lds_block_staged": ("spmv_kernels.hip", "device.hpp", "common.hpp",
                                          "analysis.hip"),
                  # the window form and its window choice
                  "V4_lds_block_windows": ("window.hip", "device.hpp", "common.hpp")}
DEFAULT_SOURCES = ("spmv_kernels.hip", "device.hpp", "common.hpp")


def kernel_source_hash(variant_name: str) -> str:
    from paper_1101_0091_amd.selector import source_hash
    return source_hash(KERNEL_SOURCES.get(variant_name, DEFAULT_SOURCES))


def stored_traffic(workload: str, variant_name: str):
    """HBM bytes per launch from committed rocprofv3 PMC runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(f"{workload}/{variant_name}")
        if e and e.get("kernel_source_hash") == kernel_source_hash(variant_name):
            return e["hbm_bytes_per_launch"]
    except (ValueError, KeyError):
        pass
    return None


def kernel_name(vname: str, sv: int = 8) -> str:
    """The product kernel of a variant (float32 storage: its float template
    or, for V6, its quads kernel)."""
    k = KERNEL_NAMES.get(vname, vname)
    if sv == 4:
        k = k.replace("<double,double", "<float,float").replace("k_sell_pairs", "k_sell_quads")
    return k


def variant_name(pkg, M) -> str:
    """The plan's variant, with V4's B-staging and window forms (kernels of
    their own) named apart."""
    v = pkg.VARIANTS[M.variant]
    if v == "V4_lds_block":
        return ("V4_lds_block", "V4_lds_block_staged", "V4_lds_block_windows")[M.v4_form]
    return v


def time_launches(fn, steps, warmup, stream, every=1):
    """HIP-event durations (ms) of every `every`-th launch, on the launch
    stream, plus the whole-region wall time (s) of all `steps` launches
    bracketed by device synchronisation. (A pair of events around every
    launch adds about 7 us of queue work to each 0.16 ms step of the
    headline product, so its timed loop samples every 8th launch.)"""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(0, steps, every)]
    t0 = time.perf_counter()
    for i in range(steps):
        if i % every == 0:
            a, b = ev[i // every]
            a.record(stream)
            fn()
            b.record(stream)
        else:
            fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in ev]
    return per, wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", type=int, default=-1, help="force a variant (default: autotune)")
    ap.add_argument("--v4-form", type=int, default=-1,
                    help="with --variant 4: force the V4 form (0 plain, 1 staged, 2 windows)")
    ap.add_argument("--workload", default="mesh", choices=["mesh", "hamiltonian"])
    ap.add_argument("--f32", action="store_true", help="FP32 storage (profiling runs)")
    ap.add_argument("--no-sell", action="store_true",
                    help="build plans without the V6 chunked copy")
    ap.add_argument("--rcm", action="store_true",
                    help="only measure the RCM-reordered workloads (host reordering ~30 s)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run the plain copy kernel on 2 x 1 GiB (counter calibration)")
    ap.add_argument("--section",
                    choices=["spmm", "batch", "batch-modes", "split", "config3-parts", "small",
                             "solvers"],
                    help="only the multi-RHS products, only the 4096-matrix batch, only "
                         "its one-launch modes, only the split product over shard sizes, or "
                         "only config 3 taken apart into its stencil and its random extras, or "
                         "only the 2D Laplacian's product and multi-RHS products, or only CG "
                         "and Lanczos on it (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import crsgen
    import paper_1101_0091_amd as pkg
    from paper_1101_0091_amd import perfmodel as pm

    global SELL
    SELL = 0 if args.no_sell else pkg.SPMV_FLAG_SELL
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.rcm:
        print(json.dumps(run_rcm(pkg, pm, dev, stream, both=True)), flush=True)
        return
    if args.calib_copy:
        n = 1 << 27  # 1 GiB of float64 read, 1 GiB written per launch
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            pkg.spmv_stream_copy(dst, src, n)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 launches of k_copy over 1 GiB")
    if args.section == "spmm":
        print(json.dumps(run_spmm_section(pkg, pm, dev, stream)), flush=True)
        return
    if args.section in ("batch", "batch-modes"):
        print(json.dumps(run_batch(pkg, pm, dev, stream, each=args.section == "batch")),
              flush=True)
        return
    if args.section == "split":
        print(json.dumps(run_split_section(pkg, pm, dev, stream)), flush=True)
        return
    if args.section == "solvers":
        print(json.dumps(run_solvers(pkg, dev)), flush=True)
        return
    if args.section == "small":
        print(json.dumps({"laplace2d_256": run_small(pkg, pm, dev, stream),
                          "spmm_laplace2d_256": run_spmm_small(pkg, pm, dev, stream)}),
              flush=True)
        return
    if args.section == "config3-parts":
        print(json.dumps(run_config3_parts(pkg, pm, dev, stream, max(20, args.steps // 4))),
              flush=True)
        return
    if args.workload == "hamiltonian":
        wname, seed = "hamiltonian_like_N6M", 2
        log("generating Hamiltonian-like matrix N=6,000,000")
        A = crsgen.hamiltonian(6_000_000, seed=seed)
    else:
        wname, seed = "mesh3d_280_permuted_N21.95M", 3
        log("generating permuted 3D stencil matrix N=21,952,000")
        A = crsgen.mesh3d(280, seed=seed)[0]
    B = crsgen.uniform_vec(A.n_cols, seed)
    flags = pkg.SPMV_SELECT_AUTOTUNE if args.variant < 0 else pkg.SPMV_FLAG_VARIANT(args.variant)
    if args.variant == 4 and args.v4_form >= 0:
        flags |= (pkg.SPMV_FLAG_V4_STAGE_OFF, pkg.SPMV_FLAG_V4_STAGE_ON,
                  pkg.SPMV_FLAG_V4_WINDOWS)[args.v4_form]
    flags |= SELL
    sv = 4 if args.f32 else 8
    vdt, bdt = (torch.float32, np.float32) if args.f32 else (torch.float64, np.float64)
    M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(bdt),
                      val_dtype=vdt, flags=flags, device=dev)
    vname = variant_name(pkg, M)
    log(f"plan ready: nnz={A.nnz} variant={vname} blocks={M.num_blocks} "
        f"sell_slots={M.sell_slots}")
    Bd = torch.from_numpy(B.astype(bdt)).to(dev)
    C = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    h = M.handle
    code = pkg.SPMV_F32 if args.f32 else pkg.SPMV_F64

    def step():
        pkg.spmv_apply(h, Bd, code, C)

    per, wall = time_launches(step, args.steps, args.warmup, stream,
                              every=8 if args.steps >= 64 else 1)
    k_ms = float(np.mean(per))
    ms_per_step = 1000.0 * wall / args.steps
    secs = ms_per_step / 1000.0
    nnz = A.nnz
    value = pm.gflops(nnz, secs)
    comp = pm.compulsory_bytes(A.n_rows, A.n_cols, nnz, 1, sv, sv)
    own = own_bytes(pkg, M, A, sv)
    achieved = own / (k_ms / 1000.0) / 1e9
    log(f"{'fp32' if args.f32 else 'fp64'}: {ms_per_step:.4f} ms/step, kernel {k_ms:.4f} ms, "
        f"{value:.1f} GFlop/s, {achieved:.1f} GB/s of the kernel's own bytes")
    traffic = None if args.f32 else stored_traffic(wname, vname)
    kappa = (None if traffic is None else
             round(pm.kappa_from_bytes(traffic, A.n_rows, A.n_cols, nnz), 3))
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFlop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.f32 else "f64",
        "data": "synthetic",
        "config": {"workload": wname, "n_rows": A.n_rows, "nnz": nnz, "seed": seed,
                   "variant": vname, "reads_caller_crs_arrays": vname != "V6_sell64",
                   "rhs": "uniform[-1,1)"},
        "eff_gbs": round(comp / secs / 1e9, 1),
        "pct_hbm_roofline": round(100.0 * comp / secs / 1e9 / HBM_PEAK, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4),
                     "traffic": traffic, "kernel": kernel_name(vname, sv),
                     "kernel_ms": round(k_ms, 5),
                     "kernel_ms_median": round(float(np.median(per)), 5),
                     "kernel_ms_min": round(float(np.min(per)), 5),
                     "algorithmic_bytes_per_launch": own,
                     "crs_compulsory_bytes_per_launch": comp,
                     "kappa_bytes_per_nnz": kappa,
                     # the counted traffic over the kernel's time: how close the
                     # bytes it actually moves come to the peak
                     "traffic_gbs": (None if traffic is None else
                                     round(traffic / (k_ms / 1000.0) / 1e9, 1)),
                     "traffic_frac": (None if traffic is None else
                                      round(traffic / (k_ms / 1000.0) / 1e9 / HBM_PEAK, 4))},
    }
    extra = {}
    if not args.no_extra:
        extra = run_extra(A, B, M, pkg, pm, dev, stream, args)
    out["extra"] = extra
    if "triad_gbs" in extra:
        # the paper's practice: performance against the measured STREAM triad
        out["pct_of_box_triad"] = round(100.0 * achieved / extra["triad_gbs"], 2)
    if not args.no_cpu_baseline:
        gpu_results = None
        if not args.f32:
            # the headline product (last timed launch) and the FP32-storage
            # product of the same matrix, for the accuracy report
            M32 = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(np.float32),
                                val_dtype=torch.float32, flags=SELL, device=dev)
            C32 = M32.apply(torch.from_numpy(B.astype(np.float32)).to(dev))
            gpu_results = (C.cpu().numpy(), C32.cpu().numpy())
            del M32, C32
        out["cpu_baseline"], out["host_node_scheme"], acc = cpu_baseline(A, B, gpu_results)
        if acc:
            out["accuracy_vs_oracle"] = acc
        out["paper_cpu_context"] = PAPER_CPU
    print(json.dumps(out), flush=True)


def own_bytes(pkg, M, A, sv, k=1):
    """Bytes the plan's product kernel must read and write once: the CRS
    compulsory bytes for kernels that read the caller's arrays, the chunked
    copy's stream plus B and C for V6."""
    from paper_1101_0091_amd import perfmodel as pm
    if M.variant == pkg.SPMV_V6_SELL64:
        return M.sell_stream_bytes + sv * A.n_cols * k + 8 * A.n_rows * k
    return pm.compulsory_bytes(A.n_rows, A.n_cols, A.nnz, k, sv, sv)


def time_create(A, pkg, dev, has_v6=True):
    """Plan creation cost: analysis only (fixed variant), analysis + selector
    network, analysis + exhaustive autotune (the selector's alternative);
    with the V6 copy where it fits the matrix."""
    import torch
    rp = torch.from_numpy(A.row_ptr).to(dev)
    ci = torch.from_numpy(A.col_idx).to(dev)
    va = torch.from_numpy(A.val).to(dev)
    out = {}
    for name, flags in (("fixed", pkg.SPMV_FLAG_VARIANT(4)), ("selector", pkg.SPMV_SELECT_DEFAULT),
                        ("autotune", pkg.SPMV_SELECT_AUTOTUNE),
                        ("fixed_v6_with_copy", pkg.SPMV_FLAG_VARIANT(6) | pkg.SPMV_FLAG_SELL),
                        ("selector_with_v6_copy", pkg.SPMV_SELECT_DEFAULT | pkg.SPMV_FLAG_SELL),
                        ("autotune_with_v6_copy", pkg.SPMV_SELECT_AUTOTUNE | pkg.SPMV_FLAG_SELL)):
        if name == "fixed_v6_with_copy" and not has_v6:
            continue
        if name.startswith("selector"):
            pkg.load_selector()
        nb = pkg.spmv_workspace_size(A.n_rows, A.n_cols, A.nnz, flags)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = pkg.spmv_create(A.n_rows, A.n_cols, A.nnz, rp, ci, va, pkg.SPMV_F64, ws, nb, flags)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            v = pkg.spmv_get_variant(h)
            pkg.spmv_destroy(h)
            best = t if best is None else min(best, t)
        out[name] = {"ms": round(best * 1e3, 3), "variant": pkg.VARIANTS[v]}
    log(f"plan creation: {out}")
    return out


def kernel_record(pkg, pm, M, A, fn, stream, sv, wname=None, steps=30):
    """Median event time of one product with the plan's current variant, its
    rate on the bytes its kernel reads (own) and on the CRS compulsory bytes."""
    import numpy as np
    per, _ = time_launches(fn, steps, 3, stream)
    t = float(np.median(per)) / 1000
    vname = variant_name(pkg, M)
    own = own_bytes(pkg, M, A, sv)
    comp = pm.compulsory_bytes(A.n_rows, A.n_cols, A.nnz, 1, sv, sv)
    rec = {"variant": vname, "kernel": kernel_name(vname, sv),
           "kernel_ms": round(t * 1e3, 5), "gflops": round(pm.gflops(A.nnz, t), 1),
           "own_bytes_per_launch": own, "own_gbs": round(own / t / 1e9, 1),
           "own_frac": round(own / t / 1e9 / HBM_PEAK, 4),
           "crs_equiv_gbs": round(comp / t / 1e9, 1),
           "crs_equiv_frac": round(comp / t / 1e9 / HBM_PEAK, 4)}
    if wname and sv == 8:
        rec["traffic"] = stored_traffic(wname, vname)
    return rec


def run_extra(A, B, M, pkg, pm, dev, stream, args):
    import numpy as np
    import torch

    import crsgen
    ex = {}
    steps = max(20, args.steps // 4)
    wname = "mesh3d_280_permuted_N21.95M" if A.n_rows != 6_000_000 else "hamiltonian_like_N6M"
    # every variant (and V4 form) on the headline matrix
    Bd = torch.from_numpy(B).to(dev)
    C = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    var_ms = {}
    v0, f0 = M.variant, M.v4_form
    for v in range(pkg.SPMV_NUM_VARIANTS):
        if v == pkg.SPMV_V6_SELL64 and M.sell_slots is None:
            continue
        M.variant = v
        for f in ((0, 1, 2) if v == 4 else (f0,)):
            M.v4_form = f
            per, _ = time_launches(lambda: pkg.spmv_apply(M.handle, Bd, pkg.SPMV_F64, C), steps,
                                   3, stream)
            var_ms[variant_name(pkg, M)] = round(float(np.median(per)), 5)
    M.variant, M.v4_form = v0, f0
    ex["variant_ms"] = var_ms
    log(f"variants: {var_ms}")
    # the timed loop reuses B, which stays in the 256 MB memory-side cache
    # between products; here a 1 GiB buffer is written before each one
    t = cold_time(lambda: pkg.spmv_apply(M.handle, Bd, pkg.SPMV_F64, C), stream)
    ex["headline_cold"] = {"ms": round(t * 1000, 5), "gflops": round(pm.gflops(A.nnz, t), 1),
                           "eff_gbs": round(pm.effective_gbs(A.n_rows, A.n_cols, A.nnz, t), 1)}
    log(f"headline cold: {ex['headline_cold']}")
    ex["plan_create_ms"] = time_create(A, pkg, dev, M.sell_slots is not None)
    # FP32 storage, FP64 accumulation
    M32 = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(np.float32),
                        val_dtype=torch.float32, flags=pkg.SPMV_SELECT_AUTOTUNE | SELL,
                        device=dev)
    B32 = torch.from_numpy(B.astype(np.float32)).to(dev)
    ex["mixed_fp32_storage"] = kernel_record(
        pkg, pm, M32, A, lambda: pkg.spmv_apply(M32.handle, B32, pkg.SPMV_F32, C), stream, 4)
    log(f"mixed: {ex['mixed_fp32_storage']}")
    del M32, B32, Bd, C
    torch.cuda.empty_cache()
    # triad ceiling
    n = 1 << 27
    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.rand(n, dtype=torch.float64, device=dev)
    c = torch.rand(n, dtype=torch.float64, device=dev)
    per, _ = time_launches(lambda: pkg.spmv_stream_triad(a, b, c, 3.0, n), 20, 3, stream)
    tt = float(np.median(per)) / 1000
    ex["triad_gbs"] = round(24 * n / tt / 1e9, 1)
    per, _ = time_launches(lambda: pkg.spmv_stream_copy(a, b, n), 20, 3, stream)
    ex["copy_gbs"] = round(16 * n / (float(np.median(per)) / 1000) / 1e9, 1)
    log(f"triad {ex['triad_gbs']} GB/s copy {ex['copy_gbs']} GB/s")
    del a, b, c
    if wname != "hamiltonian_like_N6M":
        ex["hamiltonian_like_N6M"] = run_hamiltonian(pkg, pm, dev, stream)
        ex["rcm_mesh3d_280"] = run_rcm(pkg, pm, dev, stream, A=A, B=B)["mesh3d_280_permuted"]
        ex["config3_parts"] = run_config3_parts(pkg, pm, dev, stream, steps)
        ex["split_shards_hamiltonian_like_N6M"] = run_split_section(pkg, pm, dev, stream)
    ex["spmm_laplace2d_256"] = run_spmm_small(pkg, pm, dev, stream)
    ex["batch_4096"] = run_batch(pkg, pm, dev, stream)
    ex["laplace2d_256"] = run_small(pkg, pm, dev, stream)
    ex["solvers_laplace2d_256"] = run_solvers(pkg, dev)
    return ex


def sample_rows(A):
    """A seeded sample of rows (the first and last included) and those rows of
    A as a CRS matrix of their own."""
    import numpy as np

    import crsgen
    rng = np.random.default_rng(17)
    m = min(SPMM_SAMPLE_ROWS, A.n_rows)
    rows = np.unique(np.concatenate([[0, A.n_rows - 1],
                                     rng.choice(A.n_rows, size=m, replace=False)]))
    lens = (A.row_ptr[rows + 1] - A.row_ptr[rows]).astype(np.int64)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    idx = np.concatenate([np.arange(A.row_ptr[r], A.row_ptr[r + 1]) for r in rows])
    return rows, crsgen.CRS(len(rows), A.n_cols, rp, A.col_idx[idx], A.val[idx])


def run_spmm(A, M, pkg, pm, dev, stream, ks, sv, keep=False):
    """C = A B for k right-hand sides (B and C row-major, ldb = ldc = k) with
    plan M; per k the time, FP64 GFlop/s and the fraction of 8 TB/s on the CRS
    compulsory bytes of k columns (B read once, C written once). keep: hold C
    on a row sample for the accuracy report."""
    import numpy as np
    import torch

    import crsgen
    bdt, code = (np.float32, pkg.SPMV_F32) if sv == 4 else (np.float64, pkg.SPMV_F64)
    out = {"variant": variant_name(pkg, M)}
    rows, sub = sample_rows(A) if keep else (None, None)
    for k in ks:
        Bk = torch.from_numpy(crsgen.uniform_vec(A.n_cols * k, 4).reshape(A.n_cols, k)
                              .astype(bdt)).to(dev)
        Ck = torch.empty((A.n_rows, k), dtype=torch.float64, device=dev)
        per, _ = time_launches(lambda: pkg.spmm_apply(M.handle, k, Bk, k, code, Ck, k), 20, 3,
                               stream)
        if keep:
            SPMM_SAMPLES.append({"sv": sv, "k": k, "sub": sub,
                                 "C": Ck[torch.from_numpy(rows).to(dev)].cpu().numpy()})
        t = float(np.median(per)) / 1000
        comp = pm.compulsory_bytes(A.n_rows, A.n_cols, A.nnz, k, sv, sv)
        out[str(k)] = {"us": round(t * 1e6, 1), "fp64_gflops": round(pm.gflops(A.nnz, t, k), 1),
                       "crs_equiv_frac": round(comp / t / 1e9 / HBM_PEAK, 4)}
        del Bk, Ck
    log(f"spmm: {out}")
    return out


def run_spmm_section(pkg, pm, dev, stream):
    """Only the multi-RHS products on the Hamiltonian-like matrix from the V6
    copy, FP64 and FP32 storage (the profiled command of the SpMM kernels)."""
    import numpy as np
    import torch

    import crsgen
    A = crsgen.hamiltonian(6_000_000, seed=2)
    res = {}
    for tag, vdt, bdt, sv in (("fp64", torch.float64, np.float64, 8),
                              ("fp32_storage", torch.float32, np.float32, 4)):
        M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(bdt),
                          val_dtype=vdt, flags=pkg.SPMV_FLAG_VARIANT(6) | pkg.SPMV_FLAG_SELL,
                          device=dev)
        res[tag] = run_spmm(A, M, pkg, pm, dev, stream, (2, 4, 8, 16, 32), sv)
        del M
        torch.cuda.empty_cache()
    return res


def run_split_section(pkg, pm, dev, stream):
    """Only the split product, on shards of 1/16, 1/8, 1/4 and 1/2 of the
    Hamiltonian-like matrix centred on its middle row: how the penalty of the
    second pass changes with the shard size."""
    import crsgen
    A = crsgen.hamiltonian(6_000_000, seed=2)
    B = crsgen.uniform_vec(A.n_cols, 2)
    n = A.n_rows
    res = {}
    for s in (16, 8, 4, 2):
        log(f"split shard 1/{s}")
        res[f"1/{s}"] = run_split(A, B, pkg, pm, dev, stream, n // 2 - n // (2 * s),
                                  n // 2 + n // (2 * s))
    return res


def mesh_stencil_mask(A, p, m):
    """True for the entries of the permuted mesh matrix that belong to its
    7-point stencil (p[new] = old), False for the random extras."""
    import numpy as np
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int32), np.diff(A.row_ptr))
    i = p[rows].astype(np.int64)
    del rows
    d = p[A.col_idx].astype(np.int64) - i
    x, y, z = i % m, (i // m) % m, i // (m * m)
    mm = m * m
    return ((d == 0) | ((d == 1) & (x < m - 1)) | ((d == -1) & (x > 0)) |
            ((d == m) & (y < m - 1)) | ((d == -m) & (y > 0)) |
            ((d == mm) & (z < m - 1)) | ((d == -mm) & (z > 0)))


def run_config3_parts(pkg, pm, dev, stream, steps):
    """Config 3 taken apart: its 7-point stencil alone and its ~17M random
    extras alone, each with the plan the autotuner picks, then the extras as
    a second pass adding into C after the stencil product (the split
    machinery with an empty local window), against the one-pass product."""
    import numpy as np
    import torch

    import crsgen
    m = 280
    A, p = crsgen.mesh3d(m, seed=3)
    B = crsgen.uniform_vec(A.n_cols, 3)
    st = mesh_stencil_mask(A, p, m)
    n = A.n_rows
    parts = {}
    for tag, keep in (("stencil", st), ("extras", ~st)):
        lens = np.bincount(np.repeat(np.arange(n, dtype=np.int32), np.diff(A.row_ptr))[keep],
                           minlength=n)
        rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
        parts[tag] = crsgen.CRS(n, n, rp, A.col_idx[keep], A.val[keep])
    del st
    Bd = torch.from_numpy(B).to(dev)
    res = {"nnz": A.nnz, "nnz_stencil": parts["stencil"].nnz, "nnz_extras": parts["extras"].nnz,
           "rows_with_extras": int(np.count_nonzero(np.diff(parts["extras"].row_ptr)))}
    plans = {}
    for tag, M_A in (("full", A), ("stencil", parts["stencil"]), ("extras", parts["extras"])):
        M = pkg.CRSMatrix.from_crs(M_A, flags=pkg.SPMV_SELECT_AUTOTUNE | SELL, device=dev)
        C = torch.empty(n, dtype=torch.float64, device=dev)
        log(f"config3 parts: {tag} plan {variant_name(pkg, M)}")
        res[tag] = kernel_record(pkg, pm, M, M_A,
                                 lambda: pkg.spmv_apply(M.handle, Bd, pkg.SPMV_F64, C), stream, 8,
                                 steps=steps)
        plans[tag] = (M, C)
    # two passes: stencil product, then the extras added by the split's remote pass
    E = parts["extras"]
    S = pkg.SplitMatrix(n, n, E.row_ptr, E.col_idx, E.val, 0, 0, device=dev)
    Ms, C2 = plans["stencil"]

    def two_pass():
        pkg.spmv_apply(Ms.handle, Bd, pkg.SPMV_F64, C2)
        S.apply(Bd, C2, pass_=1)
    per, _ = time_launches(two_pass, steps, 3, stream)
    res["two_pass_ms"] = round(float(np.median(per)), 5)
    per, _ = time_launches(lambda: S.apply(Bd, C2, pass_=1), steps, 3, stream)
    res["extras_second_pass_ms"] = round(float(np.median(per)), 5)
    two_pass()
    Mf, Cf = plans["full"]
    pkg.spmv_apply(Mf.handle, Bd, pkg.SPMV_F64, Cf)
    torch.cuda.synchronize()
    res["two_pass_max_rel_diff"] = float(((C2 - Cf).abs().max() / Cf.abs().max()).item())
    log(f"config3 parts: {res}")
    return res


def run_hamiltonian(pkg, pm, dev, stream):
    """The Hamiltonian-like workload (N = 6.0M, 7 symmetric offset pairs): the
    fastest kernel that reads the caller's CRS arrays (V0-V5, every V4 form)
    and V6 (the chunked copy) in FP64 and FP32 storage, each on the bytes its
    kernel reads and on the CRS compulsory bytes; multi-RHS; the split shard."""
    import numpy as np
    import torch

    import crsgen
    log("generating Hamiltonian-like matrix N=6,000,000")
    A = crsgen.hamiltonian(6_000_000, seed=2)
    B = crsgen.uniform_vec(A.n_cols, 2)
    wname = "hamiltonian_like_N6M"
    res = {"n_rows": A.n_rows, "nnz": A.nnz}
    C = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    for tag, vdt, bdt, code, sv in (("fp64", torch.float64, np.float64, pkg.SPMV_F64, 8),
                                    ("fp32_storage", torch.float32, np.float32, pkg.SPMV_F32,
                                     4)):
        M = pkg.CRSMatrix(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val.astype(bdt),
                          val_dtype=vdt, flags=pkg.SPMV_SELECT_AUTOTUNE | SELL, device=dev)
        Bd = torch.from_numpy(B.astype(bdt)).to(dev)
        at = pkg.spmv_get_autotune_times(M.handle)
        picked, pform = M.variant, M.v4_form
        rec = {"autotune_pick": variant_name(pkg, M)}
        # the fastest reader of the CRS arrays, with its fastest V4 form
        best = int(np.argmin(at[:6]))
        M.variant = best
        if best == 4:
            forms = {}
            for f in (0, 1, 2):
                M.v4_form = f
                per, _ = time_launches(lambda: pkg.spmv_apply(M.handle, Bd, code, C), 20, 3,
                                       stream)
                forms[f] = float(np.median(per))
            M.v4_form = min(forms, key=forms.get)
        rec["crs_kernel"] = kernel_record(pkg, pm, M, A,
                                          lambda: pkg.spmv_apply(M.handle, Bd, code, C), stream,
                                          sv, wname)
        if M.sell_slots is not None:
            M.variant = pkg.SPMV_V6_SELL64
            rec["v6_copy"] = kernel_record(pkg, pm, M, A,
                                           lambda: pkg.spmv_apply(M.handle, Bd, code, C), stream,
                                           sv, wname)
        M.variant, M.v4_form = picked, pform
        rec["spmm"] = run_spmm(A, M, pkg, pm, dev, stream, (1, 2, 4, 8, 16, 32), sv, keep=True)
        res[tag] = rec
        log(f"hamiltonian {tag}: {rec}")
        del M, Bd
        torch.cuda.empty_cache()
    res["split_shard"] = run_split(A, B, pkg, pm, dev, stream)
    return res


def run_split(A, B, pkg, pm, dev, stream, r0=None, r1=None):
    """The split product of eq. (2) on one shard of the workload at its real
    shape: by default rows [3N/8, 4N/8) of 8 row shards, local columns = the
    same range (the columns that shard would own). Compared with the unsplit
    product of the same rows; the model's penalty is eq. (2) / eq. (1) at
    kappa = 0."""
    import numpy as np
    import torch
    n = A.n_rows
    if r0 is None:
        r0, r1 = 3 * n // 8, 4 * n // 8
    s0, s1 = int(A.row_ptr[r0]), int(A.row_ptr[r1])
    rp = (A.row_ptr[r0:r1 + 1] - A.row_ptr[r0]).astype(np.int32)
    ci, va = A.col_idx[s0:s1], A.val[s0:s1]
    rows, nnz = r1 - r0, s1 - s0
    U = pkg.CRSMatrix(rows, n, rp, ci, va, flags=pkg.SPMV_FLAG_VARIANT(4), device=dev)
    S = pkg.SplitMatrix(rows, n, rp, ci, va, r0, r1, device=dev)
    Bd = torch.from_numpy(B).to(dev)
    C = torch.empty(rows, dtype=torch.float64, device=dev)
    res = {"rows": rows, "nnz": nnz, "nnz_local": S.nnz_local, "nnz_remote": S.nnz_remote}
    for name, fn in (("unsplit_us", lambda: U.apply(Bd, C)),
                     ("split_both_us", lambda: S.apply(Bd, C)),
                     ("split_pass0_us", lambda: S.apply(Bd, C, pass_=0)),
                     ("split_pass1_us", lambda: S.apply(Bd, C, pass_=1))):
        per, _ = time_launches(fn, 50, 5, stream)
        res[name] = round(float(np.median(per)) * 1000, 2)
    nnzr = nnz / rows
    res["measured_penalty"] = round(res["split_both_us"] / res["unsplit_us"] - 1, 4)
    res["eq2_over_eq1_penalty"] = round(pm.split_penalty(nnzr), 4)
    # GPU byte form: the split adds a second row_ptr (4 B/row) and a C read + write (16 B/row)
    base = 12 * nnz + 4 * (rows + 1) + 8 * rows + 8 * rows
    res["gpu_model_penalty"] = round((base + 4 * (rows + 1) + 16 * rows) / base - 1, 4)
    # the streams each launch must move (B gathers left out), as a rate
    b_unsplit = 12 * nnz + 4 * (rows + 1) + 8 * rows
    b_remote = 12 * S.nnz_remote + 4 * (rows + 1) + 16 * rows
    res["unsplit_stream_gbs"] = round(b_unsplit / res["unsplit_us"] / 1e3, 1)
    res["pass1_stream_gbs"] = round(b_remote / res["split_pass1_us"] / 1e3, 1)
    log(f"split: {res}")
    del U, S
    torch.cuda.empty_cache()
    return res


def run_rcm(pkg, pm, dev, stream, A=None, B=None, both=False):
    """Reverse Cuthill-McKee (host, library) on the permuted mesh (and with
    `both` the Hamiltonian-like matrix): host ordering and permutation times,
    and the reordered product P A P^T (P B) against the product as given
    (autotuned plans, kernel ms)."""
    import numpy as np
    import torch

    import crsgen
    out = {"metric": "RCM reordering effect (FP64 product, kernel ms)"}
    todo = [("mesh3d_280_permuted", lambda: crsgen.mesh3d(280, seed=3)[0], 3)]
    if both:
        todo.append(("hamiltonian_like_N6M", lambda: crsgen.hamiltonian(6_000_000, 2), 2))
    for name, make, seed in todo:
        if A is None or name != "mesh3d_280_permuted":
            A = make()
            B = crsgen.uniform_vec(A.n_cols, seed)
        t0 = time.perf_counter()
        perm = pkg.spmv_rcm_order(A.n_rows, A.row_ptr, A.col_idx, symmetric_part=True)
        t_rcm = time.perf_counter() - t0
        rp, ci, va = pkg.spmv_permute_crs(A.n_rows, A.row_ptr, A.col_idx, A.val, perm)
        t_perm = time.perf_counter() - t0 - t_rcm
        res = {"rcm_host_s": round(t_rcm, 2), "permute_host_s": round(t_perm, 2)}
        comp = pm.compulsory_bytes(A.n_rows, A.n_cols, A.nnz)
        C = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
        for tag, (r, c, v, b) in (("as_given", (A.row_ptr, A.col_idx, A.val, B)),
                                  ("rcm", (rp, ci, va, B[perm]))):
            M = pkg.CRSMatrix(A.n_rows, A.n_cols, r, c, v, flags=pkg.SPMV_SELECT_AUTOTUNE | SELL,
                              device=dev)
            Bd = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
            per, _ = time_launches(lambda: pkg.spmv_apply(M.handle, Bd, pkg.SPMV_F64, C), 30, 3,
                                   stream)
            t = float(np.median(per)) / 1000
            res[tag] = {"variant": variant_name(pkg, M), "kernel_ms": round(t * 1e3, 4),
                        "gflops": round(pm.gflops(A.nnz, t), 1),
                        "eff_gbs": round(comp / t / 1e9, 1)}
            del M, Bd
            torch.cuda.empty_cache()
        out[name] = res
        log(f"rcm {name}: {res}")
        A = B = None
    return out


def run_solvers(pkg, dev):
    """CG (graph-replayed iterations) and Lanczos on the 2D Laplacian, FP64 and
    FP32 storage: iterations, time per iteration, and the true residual
    recomputed with an FP64 product."""
    import numpy as np
    import torch

    import crsgen
    L = crsgen.laplace2d(256)
    n = L.n_rows
    # the solvers use whatever product the plan picked: autotuned over V0-V6
    fl = pkg.SPMV_SELECT_AUTOTUNE | pkg.SPMV_FLAG_SELL
    M64 = pkg.CRSMatrix.from_crs(L, flags=fl, device=dev)
    M32 = pkg.CRSMatrix(n, n, L.row_ptr, L.col_idx, L.val.astype(np.float32),
                        val_dtype=torch.float32, flags=fl, device=dev)
    xs = torch.from_numpy(crsgen.uniform_vec(n, 8)).to(dev)
    b = M64.apply(xs)
    wsb = pkg.spmv_cg_workspace_size(n)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    s = torch.cuda.Stream()
    # the same system with V0 and V4 plans: two launches per CG iteration
    # (search-direction update, product and p.Ap fused) against four
    M0 = pkg.CRSMatrix.from_crs(L, flags=pkg.SPMV_FLAG_VARIANT(0), device=dev)
    M4 = pkg.CRSMatrix.from_crs(L, flags=pkg.SPMV_FLAG_VARIANT(4), device=dev)
    res = {"variant_fp64": pkg.VARIANTS[M64.variant], "variant_fp32": pkg.VARIANTS[M32.variant]}
    for tag, M, tol in (("cg_fp64", M64, 1e-10), ("cg_fp32_storage", M32, 1e-5),
                        ("cg_fp64_v0_two_launches", M0, 1e-10),
                        ("cg_fp64_v4_four_launches", M4, 1e-10)):
        for graph in (False, True):
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, rr = pkg.spmv_cg_solve(M.handle, b, x, tol, 5000, 50, graph, ws, wsb, s)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            r = (b - M64.apply(x)).double()
            key = f"{tag}{'_graph' if graph else ''}"
            res[key] = {"iters": it, "recurrence_relres": rr,
                        "true_relres": float(torch.linalg.vector_norm(r) /
                                             torch.linalg.vector_norm(b)),
                        "us_per_iter": round(1e6 * t / max(it, 1), 2)}
    k = 300
    lb = pkg.spmv_lanczos_workspace_size(n, k)
    lws = torch.empty(lb, dtype=torch.uint8, device=dev)
    v0 = torch.from_numpy(crsgen.uniform_vec(n, 7)).to(dev)
    from scipy.linalg import eigvalsh_tridiagonal
    c = np.cos(np.pi / 257)
    for tag, M in (("lanczos_fp64", M64), ("lanczos_fp64_v0_two_launches", M0),
                   ("lanczos_fp64_v4_four_launches", M4)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        al, be = pkg.spmv_lanczos(M.handle, v0, k, lws, lb)
        t = time.perf_counter() - t0
        th = eigvalsh_tridiagonal(al, be[:-1])
        res[tag] = {"steps": k, "us_per_step": round(1e6 * t / k, 2),
                    "max_ritz_err": float(abs(th[-1] - (4 + 4 * c))),
                    "min_ritz_err": float(abs(th[0] - (4 - 4 * c)))}
    log(f"solvers: {res}")
    return res


def graph_rate(pkg, fn, stream, reps=100):
    """Seconds per call of `reps` calls captured back to back into one HIP
    graph and replayed: the GPU-side rate of a product repeated on one stream
    (as in an iterative solver), free of the per-call host cost of this
    Python driver. `fn(s)` issues one call on stream s."""
    import numpy as np
    import torch
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    pkg.spmv_graph_begin(s)
    for _ in range(reps):
        fn(s)
    g = pkg.spmv_graph_end(s)
    try:
        per, _ = time_launches(lambda: pkg.spmv_graph_launch(g, stream), 10, 2, stream)
    finally:
        torch.cuda.synchronize()
        pkg.spmv_graph_destroy(g)
    return float(np.median(per)) / 1000 / reps


def run_spmm_small(pkg, pm, dev, stream):
    """Multi-RHS on the 2D Laplacian (256^2), k = 1, 4, 8, 16, 32, FP64 and
    FP32 storage: event-timed per call, back to back, and cold."""
    import numpy as np
    import torch

    import crsgen
    L = crsgen.laplace2d(256)
    ML = pkg.CRSMatrix.from_crs(L, flags=SELL, device=dev)
    ML32 = pkg.CRSMatrix(L.n_rows, L.n_cols, L.row_ptr, L.col_idx, L.val.astype(np.float32),
                         val_dtype=torch.float32, flags=SELL, device=dev)
    spmm = {}
    for k in (1, 4, 8, 16, 32):
        Bk = torch.from_numpy(crsgen.uniform_vec(L.n_cols * k, 4).reshape(L.n_cols, k)).to(dev)
        Ck = torch.empty((L.n_rows, k), dtype=torch.float64, device=dev)
        Bk32 = Bk.float()
        def f64(s=None):
            pkg.spmm_apply(ML.handle, k, Bk, k, pkg.SPMV_F64, Ck, k, s)

        def f32(s=None):
            pkg.spmm_apply(ML32.handle, k, Bk32, k, pkg.SPMV_F32, Ck, k, s)
        per, _ = time_launches(f64, 50, 5, stream)
        t64 = float(np.median(per)) / 1000
        per, _ = time_launches(f32, 50, 5, stream)
        t32 = float(np.median(per)) / 1000
        b64, b32 = graph_rate(pkg, f64, stream), graph_rate(pkg, f32, stream)
        c64, c32 = cold_time(f64, stream), cold_time(f32, stream)
        spmm[str(k)] = {"fp64_gflops": round(pm.gflops(L.nnz, t64, k), 1),
                        "mixed_gflops": round(pm.gflops(L.nnz, t32, k), 1),
                        "fp64_graph_gflops": round(pm.gflops(L.nnz, b64, k), 1),
                        "mixed_graph_gflops": round(pm.gflops(L.nnz, b32, k), 1),
                        "fp64_cold_gflops": round(pm.gflops(L.nnz, c64, k), 1),
                        "mixed_cold_gflops": round(pm.gflops(L.nnz, c32, k), 1),
                        "fp64_us": round(t64 * 1e6, 2), "fp64_graph_us": round(b64 * 1e6, 2)}
    log(f"spmm: {spmm}")
    return spmm


def cold_time(fn, stream, reps=20):
    """Median duration (s) of fn with every cache cold: a 1 GiB buffer is
    written before each timed call."""
    import numpy as np
    import torch
    flush = torch.empty(1 << 27, dtype=torch.float64, device=stream.device)
    ts = []
    for _ in range(reps):
        flush.fill_(1.0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    del flush
    return float(np.median(ts)) / 1000


def run_small(pkg, pm, dev, stream):
    """The 2D Laplacian (256^2): fits in cache, so report warm (back to back)
    and cold (a 1 GiB buffer written between products evicts it)."""
    import numpy as np
    import torch

    import crsgen
    L = crsgen.laplace2d(256)
    M = pkg.CRSMatrix.from_crs(L, flags=pkg.SPMV_SELECT_AUTOTUNE | SELL, device=dev)
    Bd = torch.from_numpy(crsgen.uniform_vec(L.n_cols, 1)).to(dev)
    C = torch.empty(L.n_rows, dtype=torch.float64, device=dev)
    comp = pm.compulsory_bytes(L.n_rows, L.n_cols, L.nnz)
    per, _ = time_launches(lambda: pkg.spmv_apply(M.handle, Bd, pkg.SPMV_F64, C), 50, 5, stream)
    warm = float(np.median(per)) / 1000
    cold_t = cold_time(lambda: pkg.spmv_apply(M.handle, Bd, pkg.SPMV_F64, C), stream)
    g1 = graph_rate(pkg, lambda s: pkg.spmv_apply(M.handle, Bd, pkg.SPMV_F64, C, s), stream)
    res = {"variant": variant_name(pkg, M), "warm_us": round(warm * 1e6, 2),
           "graph_us": round(g1 * 1e6, 2), "graph_gflops": round(pm.gflops(L.nnz, g1), 1),
           "cold_us": round(cold_t * 1e6, 2), "warm_gflops": round(pm.gflops(L.nnz, warm), 1),
           "cold_gflops": round(pm.gflops(L.nnz, cold_t), 1),
           "warm_eff_gbs": round(comp / warm / 1e9, 1), "cold_eff_gbs": round(comp / cold_t / 1e9, 1)}
    log(f"laplace2d_256: {res}")
    return res


def run_batch(pkg, pm, dev, stream, each=True):
    """Uneven batch: 4096 seeded matrices, N log-uniform in [100, 5000]."""
    import numpy as np
    import torch

    import crsgen
    log("batch: generating 4096 small matrices")
    mats = [crsgen.family_matrix(6, i, 100, 5000)[0] for i in range(4096)]
    Bt = pkg.Batch(mats, device=dev)
    nnz, rows = int(Bt.nnz.sum()), int(Bt.n_rows.sum())
    # CRS compulsory bytes, and the bytes the tiles read: their 1- or 2-byte
    # column deltas in place of 4-byte indices, plus row_ptr, B and C
    comp = sum(pm.compulsory_bytes(m.n_rows, m.n_cols, m.nnz) for m in mats)
    own = Bt.stream_bytes + sum(4 * (m.n_rows + 1) + 8 * m.n_cols + 8 * m.n_rows for m in mats)
    B_all = torch.from_numpy(crsgen.uniform_vec(int(Bt.n_cols.sum()), 6)).to(dev)
    C_all = torch.empty(rows, dtype=torch.float64, device=dev)
    Bd, Cd, bh, ch = Bt.pointers(B_all, C_all)
    res = {"count": 4096, "rows": rows, "nnz": nnz, "tiles": Bt.ntiles,
           "crs_compulsory_bytes": comp, "own_bytes_per_launch": own}

    def rec(name, fn, steps=20):
        per, _ = time_launches(fn, steps, 3, stream)
        t = float(np.median(per)) / 1000
        res[name] = {"us": round(t * 1e6, 1), "own_gbs": round(own / t / 1e9, 1),
                     "own_frac": round(own / t / 1e9 / HBM_PEAK, 4),
                     "crs_equiv_gbs": round(comp / t / 1e9, 1),
                     "gflops": round(pm.gflops(nnz, t), 1)}

    for mode, name in ((pkg.SPMV_BATCH_DYNAMIC, "persistent_dynamic"),
                       (pkg.SPMV_BATCH_STATIC, "persistent_static"),
                       (pkg.SPMV_BATCH_TILE_GRID, "one_launch_tile_grid")):
        Bt.set_mode(mode)
        rec(name, lambda: Bt.apply(Bd, Cd))
    Bt.set_mode(pkg.SPMV_BATCH_TILE_GRID)
    # the batch (1.1 GB) exceeds the caches; cold timing shows what the
    # memory-side cache held from the previous launch
    t = cold_time(lambda: Bt.apply(Bd, Cd), stream)
    res["one_launch_tile_grid_cold"] = {"us": round(t * 1e6, 1),
                                        "own_gbs": round(own / t / 1e9, 1),
                                        "crs_equiv_gbs": round(comp / t / 1e9, 1),
                                        "gflops": round(pm.gflops(nnz, t), 1)}
    if not each:  # the one-launch modes only (counter runs)
        log(f"batch: {res}")
        return res
    rec("separate_launches_4096", lambda: Bt.apply_each(bh, ch), steps=5)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    pkg.spmv_graph_begin(s)
    Bt.apply_each(bh, ch, stream=s)
    g_each = pkg.spmv_graph_end(s)
    pkg.spmv_graph_begin(s)
    Bt.apply(Bd, Cd, stream=s)
    g_one = pkg.spmv_graph_end(s)
    Bt.set_mode(pkg.SPMV_BATCH_DYNAMIC)
    pkg.spmv_graph_begin(s)
    Bt.apply(Bd, Cd, stream=s)
    g_dyn = pkg.spmv_graph_end(s)
    Bt.set_mode(pkg.SPMV_BATCH_TILE_GRID)
    torch.cuda.synchronize()
    rec("graph_of_4096_launches", lambda: pkg.spmv_graph_launch(g_each, stream), steps=5)
    rec("graph_of_one_tile_grid_launch", lambda: pkg.spmv_graph_launch(g_one, stream))
    rec("graph_of_persistent_dynamic", lambda: pkg.spmv_graph_launch(g_dyn, stream))
    for g in (g_each, g_one, g_dyn):
        pkg.spmv_graph_destroy(g)
    log(f"batch: {res}")
    return res


def host_description():
    """Cores, sockets, NUMA nodes and model of the host (lscpu), and the CPUs
    this process may run on."""
    import subprocess
    info = {"usable_cpus": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count()}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket":
                "cores_per_socket", "Thread(s) per core": "threads_per_core",
                "NUMA node(s)": "numa_nodes", "CPU(s)": "cpus"}
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys:
                v = v.strip()
                info[keys[k.strip()]] = int(v) if v.isdigit() else v
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(A, B, gpu_results=None):
    """The oracle (single-threaded plain C) timed on one host core, and the
    paper's node scheme (OpenMP static schedule over rows, first-touch
    placement; oracle/node.c) on all the host CPUs this process may use, with
    a host triad for its fraction of STREAM. Both on the headline matrix,
    whole products repeated for a bounded sample. With the GPU's FP64 and
    FP32-storage products of the same matrix, also their error against the
    oracle's FP64 product: the FP64 one against the per-row bound
    8 nnz_row 2^-53 S_i, the FP32-storage one as max |dC| / S_i and the
    relative 2-norm (reported, not bounded)."""
    import numpy as np

    import oracle
    import oracle.node as node
    host = host_description()
    log(f"cpu baseline: timing the oracle on one core ({host})")
    reps, t = 0, 0.0
    Cref = None
    while t < 10.0 and reps < 1000:
        t0 = time.perf_counter()
        Cref, Sref = oracle.spmv(A.n_rows, A.row_ptr, A.col_idx, A.val, B)
        t += time.perf_counter() - t0
        reps += 1
    gf = 2.0 * A.nnz * reps / t / 1e9
    base = {"value": round(gf, 3), "unit": "GFlop/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} full products of the headline matrix (nnz={A.nnz}), {t:.1f} s, "
                      "single thread, includes the |a*b| magnitude sum",
            "host": host}
    log("cpu baseline: the paper's node scheme on all usable host CPUs")
    C, nreps, secs = node.spmv_bench(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.val, B,
                                     min_seconds=8.0, max_reps=200)
    triad = node.triad_gbs(1 << 27, 10)
    ngf = 2.0 * A.nnz * nreps / secs / 1e9
    from paper_1101_0091_amd import perfmodel as pm
    comp = pm.compulsory_bytes(A.n_rows, A.n_cols, A.nnz)
    gbs = comp * nreps / secs / 1e9
    scheme = {"value": round(ngf, 3), "unit": "GFlop/s", "threads": node.threads(),
              "kind": "OpenMP static rows + first touch (paper Sect. 2)",
              "eff_gbs": round(gbs, 2), "host_triad_gbs": round(triad, 2),
              "pct_of_host_triad": round(100.0 * gbs / triad, 1),
              "equals_oracle_bitwise": bool(np.array_equal(C.view(np.int64),
                                                           Cref.view(np.int64))),
              "sample": f"{nreps} full products, {secs:.1f} s"}
    log(f"node scheme: {scheme}")
    acc = None
    if gpu_results is not None:
        c64, c32 = gpu_results
        ok, worst = oracle.bound_ok(c64, Cref, A.row_ptr, Sref)
        nz = Sref > 0
        d32 = np.abs(c32 - Cref)
        acc = {"fp64_within_bound": bool(ok), "fp64_worst_error_over_bound": float(worst),
               "fp64_bitwise_equal_rows": float(np.mean(c64.view(np.int64) ==
                                                        Cref.view(np.int64))),
               "fp32_storage_max_err_over_S": float(np.max(d32[nz] / Sref[nz])),
               "fp32_storage_rel_2norm": float(np.linalg.norm(c32 - Cref) /
                                               np.linalg.norm(Cref))}
        log(f"accuracy vs the oracle: {acc}")
    if SPMM_SAMPLES:
        acc = dict(acc or {})
        acc["spmm_hamiltonian_like_N6M"] = spmm_accuracy(SPMM_SAMPLES)
    return base, scheme, acc


def spmm_accuracy(samples):
    """Per precision and k, the multi-RHS products on their row samples against
    the oracle's FP64 product of the FP64 inputs, column by column: FP64
    against the per-row bound 8 nnz_row 2^-53 S_i, FP32 storage as each
    column's max |dC| / S_i and relative 2-norm (reported, not bounded)."""
    import numpy as np

    import crsgen
    import oracle
    out = {}
    for k in sorted({s["k"] for s in samples}):
        Bh = None
        for s in samples:
            if s["k"] != k:
                continue
            sub = s["sub"]
            if Bh is None:  # the B the timed products read, in FP64
                Bh = crsgen.uniform_vec(sub.n_cols * k, 4).reshape(sub.n_cols, k)
                Cref, S = oracle.spmm(sub.n_rows, sub.row_ptr, sub.col_idx, sub.val, Bh)
            out.setdefault("fp64" if s["sv"] == 8 else "fp32_storage", {})[str(k)] = \
                spmm_column_errors(s, sub, Cref, S)
        del Bh
    out["sample"] = f"{samples[0]['sub'].n_rows} seeded rows of the N = 6.0M matrix per product"
    return out


def spmm_column_errors(s, sub, Cref, S):
    import numpy as np

    import oracle
    d = np.abs(s["C"] - Cref)
    if s["sv"] == 8:
        res = [oracle.bound_ok(s["C"][:, j], Cref[:, j], sub.row_ptr, S[:, j])
               for j in range(Cref.shape[1])]
        return {"within_bound": all(ok for ok, _ in res),
                "worst_error_over_bound": max(w for _, w in res)}
    ratio = np.where(S > 0, d / np.maximum(S, 1e-300), 0.0)
    rel = np.linalg.norm(s["C"] - Cref, axis=0) / np.linalg.norm(Cref, axis=0)
    return {"max_err_over_S_per_column": [float(f"{x:.3g}") for x in ratio.max(axis=0)],
            "rel_2norm_per_column": [float(f"{x:.3g}") for x in rel]}


if __name__ == "__main__":
    main()
