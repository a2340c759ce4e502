#!/usr/bin/env python3
"""Selected-SpMV benchmark on one MI355X.

Workload: the four FP64 bottleneck-class matrices (27-point stencil on 100^3,
uniform random 2M x 8/row, Pareto(1.5) row lengths 1M with a 200k row, short
rows 8M), x ~ U[-1, 1), generated on the device from their seeds.

One step = for every matrix: ``spmv_plan_create`` (validation),
``spmv_select`` (device features + MLP inference, falling back to the
profiling micro-benchmarks when the model is absent or unsure), format
preparation of the chosen variant, then ``--iters`` SpMVs with it (the solver
loop the selection is amortised over), and ``spmv_plan_destroy``.
``value`` = algorithmic bytes of all those SpMVs / wall time of the step.

Also reported (outside the timed steps): every variant's warm and cold
(Infinity-Cache flushed) time per matrix, the best variant, the selection
cost in SpMV-equivalents, attainable HBM bandwidth, the roofline of the
dominant kernel (HIP events on the plan stream, inside the timed steps) and
the oracle's single-thread CPU rate on the same matrices.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "selected_spmv_fp64_class_matrices_traffic.json")


def stored_traffic(kernel_names):
    """HBM bytes per launch (fetch + write) of the given kernels from the
    rocprofv3 counters stored in profiles/, or None when they were taken on
    another version of the kernels."""
    from paper_1511_02494_amd.profiling import stored_traffic as st
    return st(TRAFFIC_FILE, kernel_names)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_names(v, plan):
    """Demangled-name prefixes of the kernels one FP64 execute of variant v launches."""
    import paper_1511_02494_amd as S
    coded = "true" if plan.query(22) == S.SPMV_IDX_CODED else "false"  # 16-bit column codes
    if v == S.V_CSR_SCALAR:
        return ["void spmvsel::k_csr_scalar<double>"]
    if v == S.V_CSR_VECTOR:
        return [f"void spmvsel::k_csr_vector<double, {plan.query(1)}>"]
    if v == S.V_MERGE_PATH:
        return [f"void spmvsel::k_merge_path<double, {coded}>", "void spmvsel::k_merge_fixup<double>"]
    if v == S.V_XBLOCK_LDS:
        rows = plan.query(12)  # rows per block of the per-slice row-streaming kernel, 0 = merge path
        if plan.query(16) > 0:  # phased slices: no partial y, no slice sum
            return [f"void spmvsel::k_phased_slices<double, {plan.query(16)}, {coded}>"]
        if rows > 0:  # per-slice partials; with long rows their sums join the slice sum
            finish = "k_slice_finish" if plan.query(13) > 0 else "k_slice_sum"
            return [f"void spmvsel::k_rowstream_slices<double, {rows // 256}, {coded}>",
                    f"void spmvsel::{finish}<double, {plan.query(7)}>"]
        return ["void spmvsel::k_merge_slices<double>", "void spmvsel::k_merge_fixup_slices<double>",
                f"void spmvsel::k_slice_sum<double, {plan.query(7)}>"]
    if v == S.V_DELTA16:
        if plan.query(14) == 1:  # sliced layout, offsets of 8 or 16 bits
            o = "unsigned char" if plan.query(17) == 8 else "unsigned short"
            return [f"void spmvsel::k_sliced_d16<double, {o}>"]
        return [f"void spmvsel::k_rowstream<double, true, {plan.query(11) // 256}>"]
    return [f"void spmvsel::k_rowstream<double, false, {plan.query(2) // 256}>"]


def precision_report(S, torch, dev, mats, per, log):
    """FP32 and BF16 stored values (FP32 x, FP32 accumulation, Kahan on rows
    longer than 256) on each class matrix, with int32 indices (the FP64
    selection, or short_row where that is delta16) and with delta16 where it
    is feasible: time and GB/s against the FP64 path on the same variant, and
    max_i |y_i - y64_i| / sum_j |a_ij| |x_j| against the library's FP64 result
    (the tests pin that to the CPU oracle)."""
    import numpy as np  # noqa: F401
    out = []
    for M, rec in zip(mats, per):
        n, nnz = M["n"], M["nnz"]
        sel_v = S.VARIANTS.index(rec["selected"])
        variants = [S.V_SHORT_ROW if sel_v == S.V_DELTA16 else sel_v]
        if (M["mask"] >> S.V_DELTA16) & 1:
            variants.append(S.V_DELTA16)
        p64 = S.Plan(M["rp"], M["ci"], M["val"], M["m"], nnz=nnz)
        p64.set_variant(S.V_CSR_SCALAR)
        y64 = torch.empty(n, dtype=torch.float64, device=dev)
        p64.execute(M["x"], y64)
        pa = S.Plan(M["rp"], M["ci"], M["val"].abs(), M["m"], nnz=nnz)
        pa.set_variant(S.V_CSR_SCALAR)
        scale = torch.empty(n, dtype=torch.float64, device=dev)
        pa.execute(M["x"].abs(), scale)
        torch.cuda.synchronize()
        pa.close()
        x32 = M["x"].float()
        t64 = {v: p64.time(v, reps=20)[0] for v in variants}
        for dt, dname, tdt in ((S.SPMV_F32, "f32", torch.float32), (S.SPMV_BF16, "bf16", torch.int16)):
            vq = torch.empty(nnz + 8, dtype=tdt, device=dev)
            S.spmv_quantize(M["val"], vq, nnz, dt)
            pq = S.Plan(M["rp"], M["ci"], vq, M["m"], dt, nnz=nnz)
            for v in variants:
                tq, _ = pq.time(v, reps=20)
                pq.set_variant(v)
                yq = torch.empty(n, dtype=torch.float32, device=dev)
                pq.execute(x32, yq)
                err = (yq.double() - y64).abs()
                rel = torch.where(scale > 0, err / scale.clamp_min(1e-300), err)
                r = dict(matrix=M["name"], values=dname, variant=S.VARIANTS[v],
                         index="delta16" if v == S.V_DELTA16 else "int32",
                         us=tq * 1e6, gbs=pq.bytes(v) / tq * 1e-9,
                         f64_us=t64[v] * 1e6, f64_gbs=p64.bytes(v) / t64[v] * 1e-9,
                         speedup_vs_f64=t64[v] / tq, max_rel_err=float(rel.max()))
                out.append(r)
                log(f"  precision {M['name']:>22s} {dname:>4s} {r['variant']:>10s} "
                    f"{r['us']:7.1f} us ({r['gbs']:5.0f} GB/s; FP64 {r['f64_us']:7.1f} us) "
                    f"max err / sum|a||x| = {r['max_rel_err']:.2e}")
            pq.close()
            del vq
        p64.close()
    return out


def offset_width_report(S, torch, dev, log, scale=1):
    """delta16 (sliced) with 8-bit delta codes against 16-bit offsets (the
    paper's two delta widths, one per matrix) on two bands of 2M rows with
    30..90 nonzeros per row (generator family banded, d = 60): half width 32
    (rows capped at 65; slices span 127 columns, so 16-bit offsets would also
    fit 8 bits) and half width 200 (slices span about 460 columns; only the
    delta codes fit 8 bits), the sliced layout forced on the second.  FP64,
    FP32 and BF16 values; warm and cold time, algorithmic bytes and GB/s of
    each width, whether both give the same y, and max_i |y_i - y64_i| /
    sum_j |a_ij| |x_j| against the library's FP64 sequential CSR result."""
    n = 2_000_000 // scale
    out = []
    for w in (32, 200):
        prm = [n, 960, w]
        rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
        nnz = S.spmv_generate(S.FAMILY["banded"], prm, 9, rp)
        ci = torch.empty(nnz + 8, dtype=torch.int32, device=dev)
        val = torch.empty(nnz + 8, dtype=torch.float64, device=dev)
        S.spmv_generate(S.FAMILY["banded"], prm, 9, rp, ci, val)
        x = torch.empty(n, dtype=torch.float64, device=dev)
        S.spmv_generate_vector(n, 10, x)
        p64 = S.Plan(rp, ci, val, n, nnz=nnz)
        p64.set_variant(S.V_CSR_SCALAR)
        y64 = torch.empty(n, dtype=torch.float64, device=dev)
        p64.execute(x, y64)
        p64.close()
        pa = S.Plan(rp, ci, val.abs(), n, nnz=nnz)
        pa.set_variant(S.V_CSR_SCALAR)
        scale_v = torch.empty(n, dtype=torch.float64, device=dev)
        pa.execute(x.abs(), scale_v)
        torch.cuda.synchronize()
        pa.close()
        name = f"band_{n}_d60_w{w}"
        for dt, dname, tdt in ((S.SPMV_F64, "f64", torch.float64), (S.SPMV_F32, "f32", torch.float32),
                               (S.SPMV_BF16, "bf16", torch.int16)):
            if dt == S.SPMV_F64:
                v = val
            else:
                v = torch.empty(nnz + 16, dtype=tdt, device=dev)
                S.spmv_quantize(val, v, nnz, dt)
            plan = S.Plan(rp, ci, v, n, dt, nnz=nnz)
            h = plan.handle
            auto_layout = S.spmv_plan_query(h, 14)
            S.spmv_set_delta16_layout(h, 1)
            xin = x if dt == S.SPMV_F64 else x.float()
            r = dict(matrix=name, n=n, nnz=nnz, values=dname, automatic_layout=auto_layout,
                     span=S.spmv_plan_query(h, 18), automatic_bits=S.spmv_plan_query(h, 17))
            ys = []
            for req in (8, 16):
                S.spmv_set_delta16_offset_bits(h, req)
                t, _ = plan.time(S.V_DELTA16, reps=20)
                tc, _ = plan.time(S.V_DELTA16, reps=10, cold=True)
                by = plan.bytes(S.V_DELTA16)
                plan.set_variant(S.V_DELTA16)
                y = torch.empty(n, dtype=torch.float64 if dt == S.SPMV_F64 else torch.float32,
                                device=dev)
                plan.execute(xin, y)
                torch.cuda.synchronize()
                ys.append(y)
                r[f"bits{req}"] = dict(us=t * 1e6, cold_us=tc * 1e6, bytes=by, gbs=by / t * 1e-9,
                                       cold_gbs=by / tc * 1e-9, escapes=S.spmv_plan_query(h, 20))
            err = (ys[0].double() - y64).abs()
            rel = torch.where(scale_v > 0, err / scale_v.clamp_min(1e-300), err)
            r["same_y"] = bool(torch.equal(ys[0], ys[1]))
            r["max_rel_err"] = float(rel.max())
            out.append(r)
            b8, b16 = r["bits8"], r["bits16"]
            log(f"  codes {name} {dname:>4s} (auto {r['automatic_bits']} bits): 8-bit {b8['us']:7.1f} us "
                f"(cold {b8['cold_us']:6.1f}, {b8['bytes'] / 1e6:.0f} MB, {b8['escapes']} escapes)  "
                f"16-bit {b16['us']:7.1f} us (cold {b16['cold_us']:6.1f}, {b16['bytes'] / 1e6:.0f} MB)  "
                f"same y {r['same_y']}  max err {r['max_rel_err']:.2e}")
            plan.close()
            if dt != S.SPMV_F64:
                del v
        del rp, ci, val, x, y64, scale_v
    return out


def row_order_report(S, torch, dev, log, scale=1):
    """delta16 on three bands whose row lengths vary from d/2 to 3d/2
    (generator family banded) and whose slices are too wide to stage x in
    LDS: 4M rows with d = 8 in half width 400, 2M rows with d = 20 in half
    width 300, 1M rows with d = 100 in half width 500.  FP64; the streamed
    layout, the sliced one with rows in order and with rows sorted by length
    inside 256-row windows; warm and cold time, algorithmic bytes and slots
    of each, the automatic choice, and whether the three give the same y
    (they sum every row in column order from +0)."""
    out = []
    for n, d16, w, seed in ((4_000_000 // scale, 128, 400, 4), (2_000_000 // scale, 320, 300, 5),
                            (1_000_000 // scale, 1600, 500, 6)):
        prm = [n, d16, w]
        rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
        nnz = S.spmv_generate(S.FAMILY["banded"], prm, seed, rp)
        ci = torch.empty(nnz + 8, dtype=torch.int32, device=dev)
        val = torch.empty(nnz + 8, dtype=torch.float64, device=dev)
        S.spmv_generate(S.FAMILY["banded"], prm, seed, rp, ci, val)
        x = torch.empty(n, dtype=torch.float64, device=dev)
        S.spmv_generate_vector(n, seed + 1, x)
        plan = S.Plan(rp, ci, val, n, nnz=nnz)
        h = plan.handle
        name = f"band_{n}_d{d16 / 16:g}_w{w}"
        r = dict(matrix=name, n=n, nnz=nnz, automatic_layout=S.spmv_plan_query(h, 14),
                 automatic_sorted=S.spmv_plan_query(h, 26))
        ys = []
        for key, layout, srt in (("streamed", 0, -1), ("sliced_in_order", 1, 0), ("sliced_sorted", 1, 1)):
            S.spmv_set_delta16_layout(h, layout)
            S.spmv_set_delta16_sort(h, srt)
            t, _ = plan.time(S.V_DELTA16, reps=20)
            tc, _ = plan.time(S.V_DELTA16, reps=10, cold=True)
            by = plan.bytes(S.V_DELTA16)
            plan.set_variant(S.V_DELTA16)
            y = torch.empty(n, dtype=torch.float64, device=dev)
            plan.execute(x, y)
            ys.append(y)
            r[key] = dict(us=t * 1e6, cold_us=tc * 1e6, bytes=by, gbs=by / t * 1e-9,
                          slots=S.spmv_plan_query(h, 15) if layout == 1 else None)
        torch.cuda.synchronize()
        r["same_y"] = bool(torch.equal(ys[0], ys[1]) and torch.equal(ys[0], ys[2]))
        out.append(r)
        st, so, ss = r["streamed"], r["sliced_in_order"], r["sliced_sorted"]
        log(f"  rows {name} (auto layout {r['automatic_layout']}, sorted {r['automatic_sorted']}): "
            f"streamed {st['us']:6.1f} / {st['cold_us']:6.1f} us, in order {so['us']:6.1f} / "
            f"{so['cold_us']:6.1f} us ({so['slots'] / nnz:.2f} slots/nnz), sorted {ss['us']:6.1f} / "
            f"{ss['cold_us']:6.1f} us ({ss['slots'] / nnz:.2f} slots/nnz); same y {r['same_y']}")
        plan.close()
        del rp, ci, val, x, ys
    torch.cuda.empty_cache()
    return out


def amortization_report(S, torch, dev, mats, log, rtol=1e-8, max_iters=5000):
    """Conjugate gradients on the SPD systems of the workload (the 5-point
    Laplacian on 64^2 and the 27-point stencil on 100^3, b ~ U[-1, 1) from a
    seed): time to a solution with the learned selection against fixed
    csr_scalar (unoptimised) and csr_vector (architecture-centric), and the
    iteration count after which the selection has paid for itself."""
    import numpy as np
    systems = []
    n = 64 * 64
    rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    nnz = S.spmv_generate(0, [64, 0], 0, rp)
    ci = torch.empty(nnz + 8, dtype=torch.int32, device=dev)
    val = torch.empty(nnz + 8, dtype=torch.float64, device=dev)
    S.spmv_generate(0, [64, 0], 0, rp, ci, val)
    systems.append(dict(name="laplace2d_64^2", n=n, nnz=nnz, rp=rp, ci=ci, val=val))
    st = next(M for M in mats if M["name"].startswith("stencil27"))
    systems.append(dict(name=st["name"], n=st["n"], nnz=st["nnz"], rp=st["rp"], ci=st["ci"], val=st["val"]))
    out = []
    for sy in systems:
        b = torch.empty(sy["n"], dtype=torch.float64, device=dev)
        S.spmv_generate_vector(sy["n"], 7, b)
        rec = dict(system=sy["name"], n=sy["n"], nnz=sy["nnz"], rtol=rtol)
        for how in ("selected", "csr_scalar", "csr_vector"):
            runs = []
            for rep in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan = S.Plan(sy["rp"], sy["ci"], sy["val"], sy["n"], nnz=sy["nnz"])
                if how == "selected":
                    plan.select(S.SEL_MLP)
                else:
                    plan.set_variant(S.VARIANTS.index(how))
                t1 = time.perf_counter()
                x = torch.zeros(sy["n"], dtype=torch.float64, device=dev)
                it, rel = S.spmv_cg(plan.handle, b, x, max_iters, rtol)
                t2 = time.perf_counter()
                v = S.VARIANTS[plan.variant]
                plan.close()
                runs.append((t1 - t0, t2 - t1, it, rel, v))
            setup = float(np.median([r[0] for r in runs]))
            solve = float(np.median([r[1] for r in runs]))
            it, rel, v = runs[-1][2], runs[-1][3], runs[-1][4]
            rec[how] = dict(variant=v, setup_ms=setup * 1e3, solve_ms=solve * 1e3, iterations=it,
                            rel_resid=rel, ms_per_iteration=solve / max(it, 1) * 1e3,
                            total_ms=(setup + solve) * 1e3)
        sel = rec["selected"]
        for base in ("csr_scalar", "csr_vector"):
            bs = rec[base]
            gain = bs["ms_per_iteration"] - sel["ms_per_iteration"]
            extra = sel["setup_ms"] - bs["setup_ms"]
            rec[f"break_even_iterations_vs_{base}"] = (extra / gain if gain > 0 else None)
            rec[f"speedup_to_solution_vs_{base}"] = bs["total_ms"] / sel["total_ms"]
        log(f"  CG {sy['name']:>16s}: selected {sel['variant']} {sel['iterations']} it "
            f"{sel['total_ms']:.2f} ms (setup {sel['setup_ms']:.2f}); csr_scalar "
            f"{rec['csr_scalar']['total_ms']:.2f} ms; csr_vector {rec['csr_vector']['total_ms']:.2f} ms; "
            f"break-even vs csr_vector {rec['break_even_iterations_vs_csr_vector']}")
        out.append(rec)
    return out


def selector_eval(S, torch, dev, seeds, log, reps=5):
    """The selectors judged live on held-out matrices of the selector sweep's
    distribution (seeds never used for training or calibration): each matrix
    is generated on the device, every feasible variant timed (median of
    ``reps`` after warm-ups), and a fresh plan selected with the learned MLP
    (profiling fallback), the CART tree and the profiling cascade through
    spmv_select.  Reported per selector: hit rate within 5% of the fastest
    variant, mean regret t_pick / t_best - 1, and the median selection cost
    (spmv_select's own end-to-end time, features and fallback included,
    format preparation excluded) in SpMVs of the picked variant."""
    import numpy as np
    import synth
    from paper_1511_02494_amd import train as T
    have_clf = "dtree" in S.load_classifiers()
    sels = [("mlp", S.SEL_MLP), ("profiling", S.SEL_PROFILING)] + ([("cart", S.SEL_DTREE)] if have_clf else [])
    rows = []
    t0 = time.perf_counter()
    for seed in seeds:
        spec = synth.sweep_spec(seed)
        M = T.generate_on_device(spec, torch, dev)
        plan = S.Plan(M["rp"], M["ci"], M["val"], M["m"], nnz=M["nnz"])
        mask = plan.mask()
        times = T.time_variants(plan, mask, reps)
        plan.close()
        best = min(t for t in times if t > 0)
        row = dict(seed=seed, name=spec.name, n=M["n"], nnz=M["nnz"], best=S.VARIANTS[times.index(best)],
                   best_us=best * 1e6)
        for name, sel in sels:
            p = S.Plan(M["rp"], M["ci"], M["val"], M["m"], nnz=M["nnz"])
            info = p.select(sel)
            p.close()
            v = info["variant"]
            row[name] = dict(pick=S.VARIANTS[v], regret=times[v] / best - 1, fell_back=bool(info["fell_back"]),
                             cost_spmv=info["t_total_s"] / times[v], cost_us=info["t_total_s"] * 1e6)
        rows.append(row)
        del M
    torch.cuda.empty_cache()
    out = dict(seeds=f"{seeds[0]}..{seeds[-1]} ({len(seeds)} held-out sweep matrices)",
               seconds=time.perf_counter() - t0, rows=rows)
    for name, _ in sels:
        reg = np.array([r[name]["regret"] for r in rows])
        cost = np.array([r[name]["cost_spmv"] for r in rows])
        out[name] = dict(hit5=float(np.mean(reg <= 0.05)), mean_regret=float(reg.mean()),
                         median_cost_spmv=float(np.median(cost)),
                         cost_le20=float(np.mean(cost <= 20)),
                         fallback_rate=float(np.mean([r[name]["fell_back"] for r in rows])))
        log(f"  selector {name:>9s}: within 5% of the best on {100 * out[name]['hit5']:.1f}%, "
            f"mean regret {100 * out[name]['mean_regret']:.1f}%, median cost "
            f"{out[name]['median_cost_spmv']:.1f} SpMVs, fallback {100 * out[name]['fallback_rate']:.0f}%")
    return out


def bandwidth_bound_report(S, torch, dev, mats, read_gbs, log, scale=1):
    """The matrices of the workload that the bandwidth-bound test admits
    (working set above twice the 256 MiB Infinity Cache, fewer than 0.05
    line misses per nonzero, at least 8 nonzeros per row; decided from the
    features before timing): the 27-point stencil of the class set and three
    bands (2M rows of 30-90 nonzeros in half widths 32 and 200, 4M rows of
    8-24 nonzeros in half width 16).  For each: the learned selection, its
    warm and cold time, GB/s on its own algorithmic bytes, % of the 8 TB/s
    peak and % of the attainable streaming read measured by the probe."""
    fam = S.FAMILY["banded"]
    cands = [dict(name=M["name"], M=M, own=False) for M in mats if M["name"].startswith("stencil27")]
    for n, d16, w, seed in ((2_000_000 // scale, 960, 32, 9), (2_000_000 // scale, 960, 200, 9),
                            (4_000_000 // scale, 256, 16, 11)):
        rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
        nnz = S.spmv_generate(fam, [n, d16, w], seed, rp)
        ci = torch.empty(nnz + 8, dtype=torch.int32, device=dev)
        val = torch.empty(nnz + 8, dtype=torch.float64, device=dev)
        S.spmv_generate(fam, [n, d16, w], seed, rp, ci, val)
        x = torch.empty(n, dtype=torch.float64, device=dev)
        S.spmv_generate_vector(n, seed + 1, x)
        cands.append(dict(name=f"band_{n}_d{d16 // 16}_w{w}", own=True,
                          M=dict(rp=rp, ci=ci, val=val, x=x, n=n, m=n, nnz=nnz)))
    out = []
    for c in cands:
        M = c["M"]
        plan = S.Plan(M["rp"], M["ci"], M["val"], M["m"], nnz=M["nnz"])
        f, _ = plan.features()
        ws = 4 * (M["n"] + 1) + 12 * M["nnz"] + 16 * M["n"]
        admitted = ws > 2 * 256 * 2 ** 20 and f[10] < 0.05 and f[2] >= 8
        info = plan.select(S.SEL_MLP)
        v = info["variant"]
        tw, _ = plan.time(v, reps=20)
        tc, _ = plan.time(v, reps=10, cold=True)
        b = plan.bytes(v)
        r = dict(matrix=c["name"], n=M["n"], nnz=M["nnz"], working_set=ws, miss_per_nnz=f[10],
                 nnz_avg=f[2], admitted=admitted, selected=S.VARIANTS[v], bytes_alg=b,
                 warm_us=tw * 1e6, cold_us=tc * 1e6, warm_gbs=b / tw * 1e-9, cold_gbs=b / tc * 1e-9,
                 pct_peak_cold=100 * b / tc * 1e-9 / HBM_PEAK_GBS,
                 pct_peak_warm=100 * b / tw * 1e-9 / HBM_PEAK_GBS,
                 pct_attainable_read_cold=100 * b / tc * 1e-9 / read_gbs)
        out.append(r)
        log(f"  bandwidth-bound {'yes' if admitted else 'no '} {c['name']:>22s} {r['selected']:>10s} "
            f"cold {tc * 1e6:7.1f} us {r['cold_gbs']:5.0f} GB/s = {r['pct_peak_cold']:.1f}% of peak, "
            f"{r['pct_attainable_read_cold']:.1f}% of the probe's read; warm {r['pct_peak_warm']:.1f}%")
        plan.close()
        if c["own"]:
            del c["M"]
    torch.cuda.empty_cache()
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=100, help="SpMVs per matrix per step")
    ap.add_argument("--event-every", type=int, default=10,
                    help="bracket every k-th SpMV of the timed steps with HIP events (the "
                         "launch-duration sample of the roofline); each pair adds a few "
                         "microseconds of stream gaps, so not every launch carries one")
    ap.add_argument("--cold-reps", type=int, default=20,
                    help="cold launches per matrix for the roofline (cache flushed before each)")
    ap.add_argument("--selector", default="mlp", choices=["mlp", "profiling", "exhaustive"])
    ap.add_argument("--scale", type=int, default=1, help="divide matrix sizes (testing only)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32/BF16 report")
    ap.add_argument("--no-amortization", action="store_true", help="skip the CG report")
    ap.add_argument("--no-offset-width", action="store_true",
                    help="skip the 8- against 16-bit delta16 offset report")
    ap.add_argument("--no-row-order", action="store_true",
                    help="skip the delta16 row-order report (wide bands, rows sorted or not)")
    ap.add_argument("--cpu-seconds", type=float, default=16.0,
                    help="CPU time budget of the oracle baseline (all four matrices)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the per-variant timing table")
    ap.add_argument("--no-bandwidth-bound", action="store_true",
                    help="skip the report on the workload's bandwidth-bound matrices")
    ap.add_argument("--selector-seeds", type=int, default=64,
                    help="held-out sweep matrices (seeds 20000 + 8 k) for the live selector "
                         "evaluation; 0 skips it")
    ap.add_argument("--model", default=None)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding design); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_1511_02494_amd as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    model = args.model or S.DEFAULT_MODEL
    model_loaded = False
    if os.path.exists(model):
        S.spmv_model_load(model)
        model_loaded = True
    sel = {"mlp": S.SEL_MLP, "profiling": S.SEL_PROFILING, "exhaustive": S.SEL_EXHAUSTIVE}[args.selector]

    # ---- inputs, generated on the device from their seeds
    specs = synth.class_matrices(scale=args.scale)
    mats = []
    for sp in specs:
        fam = S.FAMILY[sp.family]
        p = sp.params
        if sp.family == "stencil3d_27":
            prm = [p["n"], 0]
            n = p["n"] ** 3
        elif sp.family == "uniform_random":
            prm = [p["n_rows"], p["n_cols"], p["per_row"]]
            n = p["n_rows"]
        elif sp.family == "powerlaw":
            prm = [p["n"], p["p16"], p["cap"], 1]
            n = p["n"]
        else:
            prm = [p["n"]]
            n = p["n"]
        m = n
        rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
        nnz = S.spmv_generate(fam, prm, sp.seed, rp)
        ci = torch.empty(nnz + 8, dtype=torch.int32, device=dev)
        val = torch.empty(nnz + 8, dtype=torch.float64, device=dev)
        S.spmv_generate(fam, prm, sp.seed, rp, ci, val)
        x = torch.empty(m, dtype=torch.float64, device=dev)
        S.spmv_generate_vector(m, sp.x_seed, x)
        y = torch.empty(n, dtype=torch.float64, device=dev)
        mats.append(dict(spec=sp, name=sp.name, n=n, m=m, nnz=nnz, rp=rp, ci=ci, val=val, x=x, y=y))
        log(f"generated {sp.name}: n={n} nnz={nnz}")
    torch.cuda.synchronize()

    read_gbs, copy_gbs = S.spmv_hbm_probe(4 << 30)
    log(f"HBM probe: read {read_gbs:.0f} GB/s, copy {copy_gbs:.0f} GB/s")

    # ---- per-variant table (outside the timed steps)
    for M in mats:
        plan = S.Plan(M["rp"], M["ci"], M["val"], M["m"], nnz=M["nnz"])
        mask = plan.mask()
        M["mask"] = mask
        M["variants"] = {}
        if not args.no_sweep:
            for v in range(6):
                if not (mask >> v) & 1:
                    continue
                warm, _ = plan.time(v, reps=20, cold=False)
                cold, _ = plan.time(v, reps=5, cold=True)
                b = plan.bytes(v)
                M["variants"][S.VARIANTS[v]] = dict(
                    warm_us=warm * 1e6, cold_us=cold * 1e6, bytes=b,
                    warm_gbs=b / warm * 1e-9, cold_gbs=b / cold * 1e-9)
                log(f"  {M['name']:>22s} {S.VARIANTS[v]:>10s} warm {warm * 1e6:8.1f} us "
                    f"({b / warm * 1e-9:6.0f} GB/s)  cold {cold * 1e6:8.1f} us "
                    f"({b / cold * 1e-9:6.0f} GB/s)")
            # the same variants reading 16-bit column codes, where they fit
            S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_CODED)
            cmask = plan.mask()
            M["coded"] = {}
            for v in (S.V_MERGE_PATH, S.V_XBLOCK_LDS, S.V_SHORT_ROW):
                if not (cmask >> v) & 1:
                    M["coded"][S.VARIANTS[v]] = None
                    continue
                warm, _ = plan.time(v, reps=20, cold=False)
                cold, _ = plan.time(v, reps=5, cold=True)
                b = plan.bytes(v)
                M["coded"][S.VARIANTS[v]] = dict(
                    warm_us=warm * 1e6, cold_us=cold * 1e6, bytes=b,
                    warm_gbs=b / warm * 1e-9, cold_gbs=b / cold * 1e-9)
                log(f"  {M['name']:>22s} {S.VARIANTS[v] + '+codes':>16s} warm {warm * 1e6:8.1f} us "
                    f"cold {cold * 1e6:8.1f} us ({b / 1e6:.1f} MB)")
            S.spmv_set_index_coding(plan.handle, S.SPMV_IDX_AUTO)
        plan.close()

    # ---- timed steps
    def one_step(record):
        out = []
        for M in mats:
            t0 = time.perf_counter()
            plan = S.Plan(M["rp"], M["ci"], M["val"], M["m"], nnz=M["nnz"])
            info = plan.select(sel)
            t1 = time.perf_counter()
            evs = []
            for it in range(args.iters):
                if record and it % args.event_every == 0:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    plan.execute(M["x"], M["y"], stream)
                    e1.record(stream)
                    evs.append((e0, e1))
                else:
                    plan.execute(M["x"], M["y"], stream)
            plan.close()  # synchronises the stream
            t2 = time.perf_counter()
            out.append(dict(info=info, t_select=t1 - t0, t_loop=t2 - t1, ev=evs))
        return out

    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()
    steps = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        steps.append(one_step(True))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start

    # ---- aggregate
    per = []
    total_bytes = 0
    for i, M in enumerate(mats):
        recs = [s[i] for s in steps]
        v = recs[-1]["info"]["variant"]
        bytes_v = None
        kern = []
        for r in recs:
            kern += [a.elapsed_time(b) * 1e-3 for a, b in r["ev"]]
        plan = S.Plan(M["rp"], M["ci"], M["val"], M["m"], nnz=M["nnz"])
        bytes_v = plan.bytes(v)
        kernels = kernel_names(v, plan)
        total_bytes += sum(plan.bytes(r["info"]["variant"]) for r in recs) * args.iters
        picks = sorted({S.VARIANTS[r["info"]["variant"]] for r in recs})
        plan.close()
        t_spmv = float(np.mean(kern))   # average launch duration (HIP events)
        sel_cost = float(np.median([r["info"]["t_total_s"] for r in recs]))
        var_tab = M["variants"]
        best = min(var_tab, key=lambda k: var_tab[k]["warm_us"]) if var_tab else None
        rec = dict(
            matrix=M["name"], n=M["n"], nnz=M["nnz"], selected=S.VARIANTS[v], picks=picks,
            kernels=kernels,
            selector_used=["profiling", "mlp", "exhaustive"][recs[-1]["info"]["selector"]],
            fell_back=bool(recs[-1]["info"]["fell_back"]),
            klass=(S.CLASSES[recs[-1]["info"]["klass"]] if recs[-1]["info"]["klass"] >= 0 else None),
            bytes_alg=bytes_v, spmv_us=t_spmv * 1e6, spmv_gbs=bytes_v / t_spmv * 1e-9,
            spmv_gflops=2 * M["nnz"] / t_spmv * 1e-9,
            pct_hbm_peak_warm=100 * bytes_v / t_spmv * 1e-9 / HBM_PEAK_GBS,
            selection_s=sel_cost, selection_spmv_equivs=sel_cost / t_spmv,
            selection_csr_scalar_equivs=(sel_cost / (var_tab["csr_scalar"]["warm_us"] * 1e-6)
                                         if "csr_scalar" in var_tab else None),
            prepare_s=float(np.median([r["info"]["t_prepare_s"] for r in recs])),
            step_matrix_s=float(np.median([r["t_select"] + r["t_loop"] for r in recs])),
        )
        rec["coded_forms"] = M.get("coded", {})
        if best:
            rec["best_variant"] = best
            rec["best_warm_gbs"] = var_tab[best]["warm_gbs"]
            rec["selected_vs_best"] = var_tab[best]["warm_us"] / var_tab[S.VARIANTS[v]]["warm_us"]
            rec["selected_cold_gbs"] = var_tab[S.VARIANTS[v]]["cold_gbs"]
            rec["pct_hbm_peak_cold"] = 100 * var_tab[S.VARIANTS[v]]["cold_gbs"] / HBM_PEAK_GBS
        per.append(rec)
        log(f"{M['name']:>22s}: {rec['selected']:>10s} {rec['spmv_us']:8.1f} us "
            f"{rec['spmv_gbs']:6.0f} GB/s; selection {sel_cost * 1e3:.2f} ms "
            f"= {rec['selection_spmv_equivs']:.1f} SpMVs")

    # ---- cold launches of each selected variant (roofline): the Infinity
    # Cache is flushed before every sampled launch, outside its event pair, on
    # the stream the kernel runs on; plus the random-gather ceiling of the
    # gather-bound selections (same gather count, x slices as the kernel's)
    for M, rec in zip(mats, per):
        v = S.VARIANTS.index(rec["selected"])
        plan = S.Plan(M["rp"], M["ci"], M["val"], M["m"], nnz=M["nnz"])
        plan.set_variant(v)
        cold = []
        for _ in range(args.cold_reps):
            S.spmv_cache_flush(stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            plan.execute(M["x"], M["y"], stream)
            e1.record(stream)
            torch.cuda.synchronize()
            cold.append(e0.elapsed_time(e1) * 1e-3)
        t_cold = float(np.mean(cold))
        rec["cold_launch_us"] = t_cold * 1e6
        rec["cold_gbs"] = rec["bytes_alg"] / t_cold * 1e-9
        rec["pct_hbm_peak_cold_live"] = 100 * rec["cold_gbs"] / HBM_PEAK_GBS
        rec["pct_attainable_read_cold"] = 100 * rec["cold_gbs"] / read_gbs
        if v in (S.V_XBLOCK_LDS, S.V_CSR_VECTOR, S.V_MERGE_PATH):
            ns = plan.query(7) if v == S.V_XBLOCK_LDS else 1
            w = -(-M["m"] // ns)
            t_g = S.spmv_gather_probe(w, 8, ns, M["nnz"])
            t_g1 = S.spmv_gather_probe(M["m"], 8, 1, M["nnz"])
            t_i = S.spmv_gather_probe2(w, 8, ns, M["nnz"], True)
            t_i1 = S.spmv_gather_probe2(M["m"], 8, 1, M["nnz"], True)
            rec["gather_ceiling"] = dict(
                gathers=M["nnz"], windows=ns, window_bytes=8 * w, probe_us=t_g * 1e6,
                probe_whole_x_us=t_g1 * 1e6, frac_warm=t_g / (rec["spmv_us"] * 1e-6),
                frac_cold=t_g / t_cold,
                indexed_probe_us=t_i * 1e6, indexed_probe_whole_x_us=t_i1 * 1e6,
                indexed_frac_warm=t_i / (rec["spmv_us"] * 1e-6), indexed_frac_cold=t_i / t_cold,
                note="probe: random 8-byte reads alone; indexed: also streaming a 4-byte column "
                     "and an 8-byte value per read, coalesced (no row sums, no y)")
            log(f"  gather ceiling {M['name']}: {M['nnz']} random 8-byte reads from {ns} x "
                f"{8 * w / 2**20:.1f} MiB windows {t_g * 1e6:.1f} us (whole x: {t_g1 * 1e6:.1f} us), "
                f"indexed {t_i * 1e6:.1f} us (whole x: {t_i1 * 1e6:.1f} us); "
                f"kernel warm {rec['spmv_us']:.1f} us, cold {t_cold * 1e6:.1f} us")
        plan.close()
        log(f"  cold {M['name']:>22s} {rec['selected']:>10s} {t_cold * 1e6:8.1f} us "
            f"({rec['cold_gbs']:6.0f} GB/s, {rec['pct_hbm_peak_cold_live']:.1f}% of peak)")

    precision = [] if args.no_precision else precision_report(S, torch, dev, mats, per, log)
    amort = [] if args.no_amortization else amortization_report(S, torch, dev, mats, log)
    offw = [] if args.no_offset_width else offset_width_report(S, torch, dev, log, args.scale)
    rows = [] if args.no_row_order else row_order_report(S, torch, dev, log, args.scale)
    seval = (selector_eval(S, torch, dev, [20000 + 8 * k for k in range(args.selector_seeds)], log)
             if args.selector_seeds > 0 else None)
    bwb = [] if args.no_bandwidth_bound else bandwidth_bound_report(S, torch, dev, mats, read_gbs, log,
                                                                    args.scale)

    value = total_bytes / t_total * 1e-9
    # the same work in flops (2 per nonzero): unlike the bytes, the same for
    # every variant, so a compressed format that moves fewer bytes shows here
    gflops = sum(2 * M["nnz"] for M in mats) * args.iters * args.steps / t_total * 1e-9
    dom = max(range(len(per)), key=lambda i: per[i]["cold_launch_us"])
    d = per[dom]
    traffic = stored_traffic(d["kernels"])
    roof = {"bound": "hbm", "achieved": d["cold_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": d["cold_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": f"{d['selected']} on {d['matrix']}",
            "bytes_per_launch": d["bytes_alg"], "launch_us": d["cold_launch_us"],
            "timing": f"cold: mean of {args.cold_reps} launches, each after an Infinity Cache "
                      "flush outside its HIP event pair, on the plan's stream",
            "warm": {"achieved": d["spmv_gbs"], "frac": d["spmv_gbs"] / HBM_PEAK_GBS,
                     "launch_us": d["spmv_us"],
                     "timing": "mean HIP-event duration of the sampled launches of the timed steps "
                               "(back to back, solver loop)"}}
    if "gather_ceiling" in d:
        roof["gather_ceiling"] = d["gather_ceiling"]

    cpu = None
    if not args.no_cpu:
        from oracle import cref
        cref.build()

        def time_oracle(threads, budget):
            tb, tt, reps, used = 0, 0.0, [], 1
            for sp, (rp, ci, val, x) in zip(specs, host_mats):
                n = len(rp) - 1
                b = 4 * (n + 1) + 12 * len(ci) + 16 * n
                k, t_m = 0, 0.0
                while t_m < budget / len(specs) or k < 3:
                    t0 = time.perf_counter()
                    _, used = cref.spmv(rp, ci, val, x, threads=threads)
                    t_m += time.perf_counter() - t0
                    k += 1
                tb += b * k
                tt += t_m
                reps.append(f"{sp.name} x{k}")
                log(f"cpu oracle ({used} threads) {sp.name}: {k} SpMVs in {t_m:.1f} s")
            return tb / tt * 1e-9, used, reps, tt

        host_mats = []
        for sp in specs:
            rp, ci, val = sp.build()
            host_mats.append((np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(ci, np.int32),
                              np.ascontiguousarray(val, np.float64),
                              np.ascontiguousarray(sp.x(len(rp) - 1), np.float64)))
        v1, _, reps1, t1 = time_oracle(False, 0.6 * args.cpu_seconds)
        vm, used, repsm, tm = time_oracle(True, 0.4 * args.cpu_seconds)
        note = ("bytes counted as for the GPU (4(N+1) + 12 NNZ + 16 N), selection not "
                "included; matrices built by the seeded host generator")
        cpu = {"value": vm, "unit": "GB/s", "cores": used, "kind": "oracle",
               "sample": "repeated SpMVs of the plain C oracle loop, OpenMP static partition "
                         f"with equal nonzeros per thread, on the four bench matrices "
                         f"({', '.join(repsm)}; {tm:.1f} s); " + note,
               "single_thread": {"value": v1, "unit": "GB/s", "cores": 1, "kind": "oracle",
                                 "sample": f"same loop, one thread ({', '.join(reps1)}; "
                                           f"{t1:.1f} s)"},
               "cpu": platform.processor() or platform.machine(), "nproc": os.cpu_count()}

    out = {
        "metric": "selected-SpMV GB/s & % HBM peak vs best variant; selection cost in SpMV-equivs",
        "value": value, "unit": "GB/s", "gflops": gflops, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_total / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "four FP64 bottleneck classes: 27-point stencil 100^3, uniform "
                               "random 2M x 8, Pareto(1.5) 1M with a 200k row, short rows 8M; "
                               f"per matrix per step: validate, select ({args.selector}), "
                               f"prepare, {args.iters} SpMVs",
                   "scale": args.scale, "iters_per_matrix": args.iters,
                   "launch_events_every": args.event_every,
                   "selector": args.selector, "model_loaded": model_loaded},
        "roofline": roof,
        "cpu_baseline": cpu,
        "hbm_probe": {"read_gbs": read_gbs, "copy_gbs": copy_gbs},
        "precision": precision,
        "amortization": amort,
        "offset_width": offw,
        "row_order": rows,
        "selector_eval": seval,
        "bandwidth_bound": bwb,
        "per_matrix": per,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
