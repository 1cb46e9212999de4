#!/usr/bin/env python3
"""Benchmark of the COO-assembly -> SpMV -> Jacobi-CG hot path on one MI355X.

Workload (the full-size 3-D case): Q1 trilinear Poisson on 127^3 hexahedra
(128^3 = 2,097,152 nodes), 64 FP64 COO triplets per element in element order
(131,096,512 triplets, int32 indices) -> 55,742,968 CSR entries.  One step
is one pass of the whole path over resident device inputs:

  1. coo_preallocate (device sort -> CSR pattern + jmap/perm)
  2. set_values_coo with the kappa = 1 values
  3. 100 x MatMult and 100 x MatMultTranspose (x ~ U[-1,1], seed 0);
     the first MatMultTranspose builds the explicit transpose
  4. Jacobi-CG to ||r|| <= 1e-10 ||b|| (b ~ U[-1,1], seed 0), then the same
     solve with every kernel bracketed by HIP events (the roofline's launch
     times; the events slow it, so the first solve's time is the one reported)
  5. set_values_coo with log-normal element diffusivity (sigma = 1, seed 1)
  6. FP64 Jacobi-CG to 1e-10 and mixed FP32/FP64 refinement to 1e-10 on
     that matrix (b ~ U[-1,1] from seed 1)

The headline value is the SpMV rate: algorithmic bytes of one MatMult
(values + column indices + row pointers + x + y) over the median event-timed
MatMult kernel.  The window walk (the default on this pattern) reads 16-bit
window columns in place of the 32-bit ones, so its own format moves 2 bytes
per entry less than those algorithmic bytes; the rate keeps the CSR figure,
and `format_bytes_per_call` gives the bytes of the format the walk reads.  The roofline object is for the kernel that dominates the
step's time, the fused SpMV + dot product of the CG iteration, timed with
HIP events on the solver's stream.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "SpMV HBM GB/s (% of peak); CG time to 1e-10 rel. resid, FP64 vs mixed"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_bytes(n: int, nnz: int, vbytes: int = 8) -> int:
    """Algorithmic bytes of y = A x for CSR: values, int32 columns, int32
    row pointers, x and y once each."""
    return nnz * (vbytes + 4) + (n + 1) * 4 + 2 * n * vbytes


def set_values_bytes(ncoo: int, nvalid: int, nnz: int) -> int:
    """Algorithmic bytes of the numeric COO stage: v once, perm once, jmap
    once, the values written once."""
    return ncoo * 8 + nvalid * 4 + (nnz + 1) * 4 + nnz * 8


def preallocate_bytes(n: int, ncoo: int, nvalid: int, nnz: int) -> int:
    """Algorithmic bytes of the symbolic stage: i and j read once; perm,
    jmap, col and rowptr written once."""
    return 8 * ncoo + 4 * nvalid + 4 * (nnz + 1) + 4 * nnz + 4 * (n + 1)


def preallocate_design_bytes(n: int, ncoo: int, nnz: int) -> int:
    """Bytes the two-stage order moves when every triplet is kept: the count
    pass reads i and j; three row passes each read their keys for the
    histogram, then keys and values and write both (the first reads i and
    writes values it does not read); the row-tile pass reads keys and
    values, gathers j and writes 64-bit keys and values; the heads passes
    read the keys (twice) and write jmap, col, rowptr, the diagonal
    positions."""
    count = 8 * ncoo
    passes = 3 * (4 * ncoo + 16 * ncoo) - 4 * ncoo
    tiles = (4 + 4 + 4 + 8 + 4) * ncoo
    heads = 2 * 8 * ncoo + 8 * nnz + 8 * (n + 1)
    return count + passes + tiles + heads


def cg_iteration_bytes(n: int, nnz: int) -> int:
    """SpMV + update (reads x p r q dinv, writes x r) + p update (reads r
    dinv p, writes p), FP64."""
    return spmv_bytes(n, nnz) + 7 * 8 * n + 4 * 8 * n


DOMINANT_SOURCES = ("paper_2406_08646_amd/csrc/cg.hip", "paper_2406_08646_amd/csrc/solver_core.hpp",
                    "paper_2406_08646_amd/csrc/spmv_core.hpp", "paper_2406_08646_amd/csrc/device.hpp",
                    "paper_2406_08646_amd/csrc/common.hpp", "paper_2406_08646_amd/csrc/spmv.hip",
                    "paper_2406_08646_amd/csrc/window.hip")
WALKS = {1: "vector", 2: "stream", 3: "dma", 4: "window"}
TRAFFIC_SUMMARY = "profiles/traffic_counters_q1_3d_127.md"


def kernel_source_hash() -> str:
    """Hash of the sources that define the dominant kernel; a counter
    summary taken from other sources is stale."""
    import hashlib

    h = hashlib.sha1()
    for rel in DOMINANT_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is missing or was taken from other sources."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    want = kernel_source_hash()
    with open(path) as f:
        for line in f:
            if line.startswith("dominant-kernel-traffic:"):
                fields = dict(kv.split("=") for kv in line.split(":", 1)[1].split())
                if fields.get("source") == want:
                    return int(fields["bytes_per_launch"])
    return None


def host_cpu():
    """CPU model name, logical CPU count and socket count of this host."""
    model, sockets = "", set()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and not model:
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("physical id"):
                    sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    return model or platform.processor() or "", os.cpu_count(), max(1, len(sockets))


EXTRAS = ("ceilings", "spmm16", "vec_coo", "cg_forms", "c1_cg", "one_gpu_share", "sync_vs_async",
          "batched64", "batched_small", "nonsymmetric_batch64", "lbfgs", "gradient256")


def run_extras(spx, W, torch, np, dev, prob, x_np, b_np, log, only=None):
    """Measurements of the other workloads, outside the timed steps: the
    16-RHS SpMM and the single-reduction vs textbook CG on the full 3-D
    matrix, the 64-system batch (batched vs ensemble vs one solve per
    system) and the 256^2 gradient."""
    from paper_2406_08646_amd import autograd as AG, autotune

    out = {}
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    want = lambda name: only is None or name in only
    shared = {}

    def main_matrix():
        """The full 3-D matrix, assembled once for the sections that use it."""
        if "A" not in shared:
            M = spx.coo_preallocate(prob.n, d(prob.i), d(prob.j))
            M.set_values_coo(d(prob.v))
            shared["A"] = M
        return shared["A"]

    def timed(fn, reps=1):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            best = ms if best is None else min(best, ms)
        return best, r

    def ev_ms(fn, reps=20):
        for _ in range(3):
            fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for s_, e_ in evs:
            s_.record()
            fn()
            e_.record()
        torch.cuda.synchronize()
        return statistics.median(s_.elapsed_time(e_) for s_, e_ in evs)

    # ---- what this device sustains: the library's copy and read references over
    # 2 GiB (HBM) and a copy over 2 x 96 MiB (resident in the 256 MB last-level cache)
    if want("ceilings"):
        big = torch.ones(2**28, dtype=torch.float64, device=dev)
        big2 = torch.empty_like(big)
        parts = torch.empty(2048, dtype=torch.float64, device=dev)
        copy_ms = ev_ms(lambda: spx.stream_copy(big, big2))
        read_ms = ev_ms(lambda: spx.stream_sum(big, parts))
        del big, big2
        small = torch.ones(12 * 2**20, dtype=torch.float64, device=dev)
        small2 = torch.empty_like(small)
        mall_ms = ev_ms(lambda: spx.stream_copy(small, small2), reps=50)
        del small, small2
        out["ceilings"] = {"copy_hbm_gbs": round(2 * 8 * 2**28 / (copy_ms * 1e-3) / 1e9, 1),
                           "read_hbm_gbs": round(8 * 2**28 / (read_ms * 1e-3) / 1e9, 1),
                           "copy_llc_resident_gbs": round(2 * 8 * 12 * 2**20 / (mall_ms * 1e-3) / 1e9, 1)}
        log(f"ceilings: {out['ceilings']}")

    # ---- multi-RHS SpMM on the full 3-D matrix
    if want("spmm16"):
        A = main_matrix()
        X = d(W.spmm_rhs(prob.n, 16))
        Y = torch.empty_like(X)
        spmm_tune = autotune.tune_spmm(A, X)
        for _ in range(3):
            A.spmm(X, Y)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
        for s_, e_ in ev:
            s_.record()
            A.spmm(X, Y)
            e_.record()
        torch.cuda.synchronize()
        spmm_ms = statistics.median(s_.elapsed_time(e_) for s_, e_ in ev)
        nnz = A.nnz
        spmm_bytes = nnz * 12 + (prob.n + 1) * 4 + 2 * 16 * 8 * prob.n
        xd, yd = d(x_np), torch.empty(prob.n, dtype=torch.float64, device=dev)
        for s_, e_ in ev:
            s_.record()
            A.matmult(xd, yd)
            e_.record()
        torch.cuda.synchronize()
        mv_ms = statistics.median(s_.elapsed_time(e_) for s_, e_ in ev)
        # what the staged kernel reads: values and 2-byte list positions per
        # entry, row bounds, one list per tile (192, 320 or 640 ints for 16-,
        # 32- and 64-row tiles), X and Y
        tr = spmm_tune["rows"]
        list_ints = {16: 192, 32: 320, 64: 640}[tr]
        spmm_format_bytes = (nnz * 10 + (prob.n + 1) * 4 + (prob.n + tr - 1) // tr * 4 * list_ints
                             + 2 * 16 * 8 * prob.n)
        out["spmm16"] = {"ms": round(spmm_ms, 4), "bytes": spmm_bytes,
                         "gbs": round(spmm_bytes / (spmm_ms * 1e-3) / 1e9, 1),
                         "format_bytes": spmm_format_bytes,
                         "format_gbs": round(spmm_format_bytes / (spmm_ms * 1e-3) / 1e9, 1),
                         "kernel": "k_spmm_rowset",
                         "tile_rows": spmm_tune["rows"],
                         "tile_rows_ms": {str(k): round(v, 4) for k, v in spmm_tune["all"].items()},
                         "vs_16_spmv": round(16 * mv_ms / spmm_ms, 2)}
        log(f"spmm16: {spmm_ms:.3f} ms")
        del X, Y

    # ---- COO vector assembly: the element load vector of the same mesh (8 contributions
    # per element, one per local node, in element order)
    if want("vec_coo"):
        iv = d(np.ascontiguousarray(prob.i.reshape(-1, prob.nloc, prob.nloc)[:, :, 0].reshape(-1)))
        vv = d(W.spmm_rhs(iv.numel(), 1).reshape(-1))
        xv = torch.zeros(prob.n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        V = spx.vec_coo_preallocate(prob.n, iv)
        torch.cuda.synchronize()
        pre_ms = (time.perf_counter() - t0) * 1e3
        info = V.get_info()
        for _ in range(3):
            V.set_values_coo(vv, xv)
        evv = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
        for s_, e_ in evv:
            s_.record()
            V.set_values_coo(vv, xv)
            e_.record()
        torch.cuda.synchronize()
        vset_ms = statistics.median(s_.elapsed_time(e_) for s_, e_ in evv)
        ncv, nuq = iv.numel(), int(info["nunique"])
        vbytes = ncv * 8 + ncv * 4 + (nuq + 1) * 4 + nuq * 8 + nuq * 4
        out["vec_coo"] = {"ncoo": ncv, "entries": nuq, "preallocate_ms": round(pre_ms, 3),
                          "set_values_ms": round(vset_ms, 4), "bytes": vbytes,
                          "gbs": round(vbytes / (vset_ms * 1e-3) / 1e9, 1)}
        log(f"vec_coo: {ncv} triplets -> {nuq} entries, set_values {vset_ms:.3f} ms")
        V.destroy()
        del iv, vv, xv

    # ---- single-reduction vs textbook CG on the same matrix and b
    if want("cg_forms"):
        A = main_matrix()
        b_d = d(b_np)
        forms = {}
        for name, variant in (("textbook", 0), ("single_reduction", 1), ("pipelined", 2)):
            A.set_option(spx.OPT_CG_VARIANT, variant)
            A.cg_solve(b_d, rtol=1e-10)  # warm
            A.set_option(spx.OPT_PROFILE, 1)
            A.reset_profile()
            A.cg_solve(b_d, rtol=1e-10)
            prof = A.get_profile()
            A.set_option(spx.OPT_PROFILE, 0)
            ms_plain, r2 = timed(lambda: A.cg_solve(b_d, rtol=1e-10), reps=2)
            forms[name] = {"ms": round(ms_plain, 2), "iters": r2.iters, "relres": r2.relres,
                           "status": r2.status,
                           "ms_per_iter": round(ms_plain / max(1, r2.iters), 4),
                           "kernels_ms": {k: round(v[0] / max(1, v[1]), 4)
                                          for k, v in prof.items() if v[1] > 0}}
        A.set_option(spx.OPT_CG_VARIANT, 0)
        forms["speedup"] = round(forms["textbook"]["ms_per_iter"]
                                 / forms["single_reduction"]["ms_per_iter"], 3)
        forms["pipelined_speedup"] = round(forms["textbook"]["ms_per_iter"]
                                           / forms["pipelined"]["ms_per_iter"], 3)
        out["cg_forms"] = forms
        log(f"cg forms: textbook {forms['textbook']['ms_per_iter']} ms/it, single reduction "
            f"{forms['single_reduction']['ms_per_iter']} ms/it, pipelined "
            f"{forms['pipelined']['ms_per_iter']} ms/it")
        shared.pop("A").destroy()

    # ---- C1 (2-D Q1, 63^2 elements): CG latency per iteration, grid path and one workgroup
    if want("c1_cg"):
        p1, _, b1 = W.config1()
        A1 = spx.coo_preallocate(p1.n, d(p1.i), d(p1.j))
        A1.set_values_coo(d(p1.v))
        b1d = d(b1)
        c1 = {"n": p1.n, "nnz": A1.nnz}
        for mode, form, tag in ((0, 0, "grid"), (2, 0, "one_workgroup"),
                                (0, 1, "single_reduction"), (0, 2, "pipelined")):
            A1.set_option(spx.OPT_SMALL_SOLVE, mode)
            A1.set_option(spx.OPT_CG_VARIANT, form)
            A1.cg_solve(b1d, rtol=1e-8)
            ms, r = timed(lambda: A1.cg_solve(b1d, rtol=1e-8), reps=3)
            c1[tag] = {"ms": round(ms, 3), "iters": r.iters, "relres": r.relres,
                       "us_per_iter": round(1e3 * ms / max(1, r.iters), 2)}
        A1.set_option(spx.OPT_CG_VARIANT, 0)
        out["c1_cg"] = c1
        log(f"C1 CG: {c1}")
        A1.destroy()

    # ---- one GPU's share of an 8-way row-slab partition of the 3-D matrix: rows of a
    # 128 x 128 x 16 slab as the library's diagonal block (columns in the slab) and
    # compressed off-diagonal block (the two neighbouring planes' ghost columns, only
    # the rows that touch them), assembled from the whole COO stream
    if want("one_gpu_share"):
        M = prob.grid + 1
        plane = M * M
        lo_r, hi_r = 48 * plane, 64 * plane
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S = spx.split_preallocate(prob.n, lo_r, hi_r, d(prob.i), d(prob.j))
        torch.cuda.synchronize()
        pre_ms = (time.perf_counter() - t0) * 1e3
        v_d = d(prob.v)
        S.set_values_coo(v_d)
        x_full = d(x_np)
        x_loc = x_full[lo_r:hi_r].contiguous()
        x_gh = S.gather_ghosts(x_full)
        y_loc = torch.empty_like(x_loc)
        Dg, Og = S.diag, S.offdiag
        dms = ev_ms(lambda: Dg.matmult(x_loc, y_loc))
        tms = ev_ms(lambda: S.matmult(x_loc, x_gh, y_loc))
        gms = ev_ms(lambda: S.gather_ghosts(x_full, x_gh))
        sms = ev_ms(lambda: S.set_values_coo(v_d))
        ng = hi_r - lo_r
        dnnz, onnz = Dg.nnz, Og.nnz
        dbytes = dnnz * 12 + (ng + 1) * 4 + 16 * ng
        tbytes = dbytes + onnz * 12 + (S.nrows_offdiag + 1) * 4 + 8 * S.nghost \
            + 4 * S.nrows_offdiag + 16 * S.nrows_offdiag
        out["one_gpu_share"] = {"rows": ng, "diag_nnz": dnnz, "offdiag_nnz": onnz,
                                "ghosts": S.nghost, "offdiag_rows": S.nrows_offdiag,
                                "remote_triplets": S.nremote,
                                "split_preallocate_ms": round(pre_ms, 2),
                                "set_values_ms": round(sms, 4),
                                "diag_ms": round(dms, 4),
                                "diag_gbs": round(dbytes / (dms * 1e-3) / 1e9, 1),
                                "product_ms": round(tms, 4),
                                "product_gbs": round(tbytes / (tms * 1e-3) / 1e9, 1),
                                "offdiag_add_ms": round(tms - dms, 4),
                                "ghost_gather_ms": round(gms, 4),
                                "halo_bytes_per_neighbour": plane * 8,
                                "note": "the halo exchange the off-diagonal product waits for "
                                        "is not built (one GPU); the ghost gather stands in"}
        log(f"one-GPU share: {out['one_gpu_share']}")
        S.destroy()
        del v_d, x_full, x_loc, x_gh, y_loc

    # ---- host poll after every iteration ("synchronous") vs every 20 ("asynchronous"),
    # time per iteration against the number of nonzeros, CG and TFQMR
    if want("sync_vs_async"):
        curve = []
        for dim, N in ((2, 16), (2, 32), (2, 64), (2, 128), (2, 256), (2, 512), (3, 24), (3, 48),
                       (3, 96)):
            pq = W.q1_poisson(N, dim)
            Aq = spx.coo_preallocate(pq.n, d(pq.i), d(pq.j))
            Aq.set_values_coo(d(pq.v))
            Aq.set_option(spx.OPT_CG_VARIANT, 0)  # the textbook form on both sides of the comparison
            bq = torch.ones(pq.n, dtype=torch.float64, device=dev)
            one = spx.batch_create([Aq])
            row = {"dim": dim, "grid": N, "n": pq.n, "nnz": Aq.nnz}
            for ce, tag in ((1, "sync"), (20, "async")):
                Aq.cg_solve(bq, rtol=0.0, maxit=20, check_every=ce)
                ms, r = timed(lambda: Aq.cg_solve(bq, rtol=0.0, maxit=200, check_every=ce), reps=3)
                row[f"cg_{tag}_us_per_iter"] = round(1e3 * ms / max(1, r.iters), 2)
                one.batch_tfqmr(bq, rtol=0.0, maxit=20, check_every=ce)
                ms, r = timed(lambda: one.batch_tfqmr(bq, rtol=0.0, maxit=400, check_every=ce), reps=3)
                row[f"tfqmr_{tag}_us_per_halfstep"] = round(1e3 * ms / max(1, r[1][0]), 2)
            xq = torch.zeros_like(bq)
            Aq.set_option(spx.OPT_GRAPH, 1)
            Aq.cg_solve(bq, x=xq.zero_(), rtol=0.0, maxit=200, check_every=20)  # capture
            ms, r = timed(lambda: Aq.cg_solve(bq, x=xq.zero_(), rtol=0.0, maxit=200, check_every=20),
                          reps=3)
            Aq.set_option(spx.OPT_GRAPH, 0)
            row["cg_async_graph_us_per_iter"] = round(1e3 * ms / max(1, r.iters), 2)
            row["cg_async_speedup"] = round(row["cg_sync_us_per_iter"] / row["cg_async_us_per_iter"], 2)
            row["cg_graph_speedup"] = round(row["cg_sync_us_per_iter"] / row["cg_async_graph_us_per_iter"], 2)
            row["tfqmr_async_speedup"] = round(row["tfqmr_sync_us_per_halfstep"]
                                               / row["tfqmr_async_us_per_halfstep"], 2)
            curve.append(row)
            log(f"async curve nnz={Aq.nnz}: cg {row['cg_sync_us_per_iter']} vs "
                f"{row['cg_async_us_per_iter']} (graph {row['cg_async_graph_us_per_iter']}) us/it, tfqmr {row['tfqmr_sync_us_per_halfstep']} vs "
                f"{row['tfqmr_async_us_per_halfstep']} us/half-step")
            one.destroy()
            Aq.destroy()
        out["sync_vs_async"] = {"points": curve,
                                "note": "host polls the device stop flag after every iteration (sync) "
                                        "or every 20 (async, also with each chunk replayed as one HIP "
                                        "graph); 200 CG iterations / 400 TFQMR half-steps with rtol = 0, "
                                        "time per iteration"}

    # ---- 64-system batch
    if want("batched64"):
        probs, bs = W.config4()
        mats = [spx.coo_preallocate(p.n, d(p.i), d(p.j)) for p in probs]
        for m, p in zip(mats, probs):
            m.set_values_coo(d(p.v))
        batch = spx.batch_create(mats)
        bvec = d(np.concatenate(bs))
        # the tuner's full default grid: the persistent form and 27 shapes of
        # the per-phase form (workgroups, row walk, weight exponent)
        cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        best = autotune.tune_batch(batch, bvec, rtol=1e-8,
                                   candidates=autotune.default_candidates(cus))
        kw = dict(blocks=best["blocks"], rows_per_tile=best["rows_per_tile"],
                  weight_exponent=best["weight_exponent"], persistent=best["persistent"])
        bt_ms, (xb, iters, relres, st) = timed(lambda: batch.batch_cg(bvec, rtol=1e-8, **kw), reps=3)
        # the persistent form on this batch: its largest system (512^2 rows)
        # alone on one workgroup sets the time
        pc_ms, (_, _, _, pc_st) = timed(lambda: batch.batch_cg(bvec, rtol=1e-8, persistent=1))
        work = sum(it * cg_iteration_bytes(p.n, m.nnz) for it, p, m in zip(iters, probs, mats))
        # one solve per system
        seq_ms, _ = timed(lambda: [m.cg_solve(d_b, rtol=1e-8) for m, d_b in
                                   zip(mats, [d(b) for b in bs])])
        # ensemble: the block-diagonal stack as one system (one global norm)
        offs = np.cumsum([0] + [p.n for p in probs])
        ei = np.concatenate([p.i + o for p, o in zip(probs, offs)]).astype(np.int32)
        ej = np.concatenate([p.j + o for p, o in zip(probs, offs)]).astype(np.int32)
        ev_ = np.concatenate([p.v for p in probs])
        E = spx.coo_preallocate(int(offs[-1]), d(ei), d(ej))
        E.set_values_coo(d(ev_))
        ens_ms, ens = timed(lambda: E.cg_solve(bvec, rtol=1e-8), reps=2)
        out["batched64"] = {"ms": round(bt_ms, 2), "solves_per_s": round(64 / (bt_ms * 1e-3), 1),
                            "status": st, "max_relres": max(relres), "iters_max": max(iters),
                            "iters_min": min(iters), "work_bytes": work,
                            "gbs": round(work / (bt_ms * 1e-3) / 1e9, 1), "tuning": best,
                            "tuning_candidates": len(autotune.default_candidates(cus)),
                            "sequential_ms": round(seq_ms, 2), "ensemble_ms": round(ens_ms, 2),
                            "ensemble_iters": ens.iters,
                            "speedup_vs_ensemble": round(ens_ms / bt_ms, 2),
                            "speedup_vs_sequential": round(seq_ms / bt_ms, 2),
                            "persistent_ms": round(pc_ms, 2), "persistent_status": pc_st}
        log(f"batched: {bt_ms:.2f} ms, ensemble {ens_ms:.2f} ms, sequential {seq_ms:.2f} ms")
        del batch, mats, E

    # ---- many small systems (the batched solvers' own regime): the persistent
    # launch (a workgroup per system, from a queue) vs one launch per phase vs
    # the ensemble
    if want("batched_small"):
        nsm, lo_s, hi_s = 2048, 16, 64
        probs_s, bs_s = W.config4(nsys=nsm, lo=lo_s, hi=hi_s, seed=5)
        mats_s = [spx.coo_preallocate(p.n, d(p.i), d(p.j)) for p in probs_s]
        for m, p in zip(mats_s, probs_s):
            m.set_values_coo(d(p.v))
        batch_s = spx.batch_create(mats_s)
        bvec_s = d(np.concatenate(bs_s))
        ms_p, (xp_, it_p, rel_p, st_p) = timed(lambda: batch_s.batch_cg(bvec_s, rtol=1e-8, persistent=1),
                                              reps=3)
        ms_f, (xf_, it_f, rel_f, st_f) = timed(lambda: batch_s.batch_cg(bvec_s, rtol=1e-8, persistent=-1),
                                              reps=3)
        offs_s = np.cumsum([0] + [p.n for p in probs_s])
        E_s = spx.coo_preallocate(int(offs_s[-1]),
                                  d(np.concatenate([p.i + o for p, o in zip(probs_s, offs_s)]).astype(np.int32)),
                                  d(np.concatenate([p.j + o for p, o in zip(probs_s, offs_s)]).astype(np.int32)))
        E_s.set_values_coo(d(np.concatenate([p.v for p in probs_s])))
        ms_e, ens_s = timed(lambda: E_s.cg_solve(bvec_s, rtol=1e-8), reps=2)
        work_s = sum(it * cg_iteration_bytes(p.n, m.nnz) for it, p, m in zip(it_p, probs_s, mats_s))
        out["batched_small"] = {
            "systems": nsm, "sides": [lo_s, hi_s], "rows": int(offs_s[-1]),
            "persistent_ms": round(ms_p, 2), "persistent_status": st_p,
            "persistent_solves_per_s": round(nsm / (ms_p * 1e-3), 1),
            "persistent_gbs": round(work_s / (ms_p * 1e-3) / 1e9, 1),
            "per_phase_ms": round(ms_f, 2), "per_phase_status": st_f,
            "ensemble_ms": round(ms_e, 2), "ensemble_iters": ens_s.iters,
            "max_relres": max(max(rel_p), max(rel_f)), "iters_max": max(it_p),
            "persistent_vs_per_phase": round(ms_f / ms_p, 2),
            "persistent_vs_ensemble": round(ms_e / ms_p, 2)}
        log(f"batched small ({nsm} systems): persistent {ms_p:.2f} ms, per phase {ms_f:.2f} ms, "
            f"ensemble {ms_e:.2f} ms")
        del batch_s, mats_s, E_s
        # the non-symmetric methods on as many convection-diffusion systems
        probs_n, bs_n = W.config6(nsys=nsm, lo=lo_s, hi=hi_s, seed=6)
        mats_n = [spx.coo_preallocate(p.n, d(p.i), d(p.j)) for p in probs_n]
        for m, p in zip(mats_n, probs_n):
            m.set_values_coo(d(p.v))
        batch_n = spx.batch_create(mats_n)
        bvec_n = d(np.concatenate(bs_n))
        offs_n = np.cumsum([0] + [p.n for p in probs_n])
        E_n = spx.coo_preallocate(int(offs_n[-1]),
                                  d(np.concatenate([p.i + o for p, o in zip(probs_n, offs_n)]).astype(np.int32)),
                                  d(np.concatenate([p.j + o for p, o in zip(probs_n, offs_n)]).astype(np.int32)))
        E_n.set_values_coo(d(np.concatenate([p.v for p in probs_n])))
        ens_n = spx.batch_create([E_n])
        for method in ("tfqmr", "bicg"):
            fn = "batch_" + method
            getattr(batch_n, fn)(bvec_n, rtol=1e-8, persistent=-1)  # warm (BiCG builds the transposes)
            ms_pn, (_, it_pn, rel_pn, st_pn) = timed(
                lambda: getattr(batch_n, fn)(bvec_n, rtol=1e-8, persistent=1), reps=3)
            ms_fn, (_, it_fn, rel_fn, st_fn) = timed(
                lambda: getattr(batch_n, fn)(bvec_n, rtol=1e-8, persistent=-1), reps=3)
            ms_en, (_, it_en, _, st_en) = timed(lambda: getattr(ens_n, fn)(bvec_n, rtol=1e-8), reps=2)
            out["batched_small"][method] = {
                "persistent_ms": round(ms_pn, 2), "persistent_status": st_pn,
                "per_phase_ms": round(ms_fn, 2), "per_phase_status": st_fn,
                "ensemble_ms": round(ms_en, 2), "ensemble_iters": it_en[0], "ensemble_status": st_en,
                "max_relres": max(max(rel_pn), max(rel_fn)), "iters_max": max(it_pn),
                "persistent_vs_per_phase": round(ms_fn / ms_pn, 2),
                "persistent_vs_ensemble": round(ms_en / ms_pn, 2)}
            log(f"batched small {method}: persistent {ms_pn:.2f} ms, per phase {ms_fn:.2f} ms, "
                f"ensemble {ms_en:.2f} ms")
        del batch_n, mats_n, E_n, ens_n

    # ---- 64-system non-symmetric batch: batched TFQMR / BiCG vs ensemble vs one per system
    if want("nonsymmetric_batch64"):
        probs6, bs6 = W.config6()
        mats6 = [spx.coo_preallocate(p.n, d(p.i), d(p.j)) for p in probs6]
        for m, p in zip(mats6, probs6):
            m.set_values_coo(d(p.v))
        batch6 = spx.batch_create(mats6)
        bvec6 = d(np.concatenate(bs6))
        offs6 = np.cumsum([0] + [p.n for p in probs6])
        E6 = spx.coo_preallocate(int(offs6[-1]),
                                 d(np.concatenate([p.i + o for p, o in zip(probs6, offs6)]).astype(np.int32)),
                                 d(np.concatenate([p.j + o for p, o in zip(probs6, offs6)]).astype(np.int32)))
        E6.set_values_coo(d(np.concatenate([p.v for p in probs6])))
        ens6 = spx.batch_create([E6])
        singles = [spx.batch_create([m]) for m in mats6]
        b_parts = [d(b) for b in bs6]
        nonsym = {}
        for method in ("tfqmr", "bicg"):
            fn = "batch_" + method
            getattr(batch6, fn)(bvec6, rtol=1e-8)  # warm (BiCG builds the transposes)
            ms_b, (xb, it_b, rel_b, st_b) = timed(lambda: getattr(batch6, fn)(bvec6, rtol=1e-8), reps=3)
            ms_e, (xe, it_e, rel_e, st_e) = timed(lambda: getattr(ens6, fn)(bvec6, rtol=1e-8), reps=2)
            ms_s, _ = timed(lambda: [getattr(sb, fn)(bp, rtol=1e-8) for sb, bp in zip(singles, b_parts)])
            nonsym[method] = {"ms": round(ms_b, 2), "solves_per_s": round(64 / (ms_b * 1e-3), 1),
                              "status": st_b, "max_relres": max(rel_b), "iters_max": max(it_b),
                              "iters_min": min(it_b), "ensemble_ms": round(ms_e, 2),
                              "ensemble_iters": it_e[0], "ensemble_status": st_e,
                              "sequential_ms": round(ms_s, 2),
                              "speedup_vs_ensemble": round(ms_e / ms_b, 2),
                              "speedup_vs_sequential": round(ms_s / ms_b, 2)}
            log(f"nonsymmetric batch {method}: {ms_b:.2f} ms, ensemble {ms_e:.2f} ms, "
                f"sequential {ms_s:.2f} ms")
        nonsym["iteration_unit"] = {"tfqmr": "half-steps (one product with A)",
                                    "bicg": "BiCG steps (one product with A and one with A^T)"}
        out["nonsymmetric_batch64"] = nonsym
        del batch6, mats6, E6, ens6, singles

    # ---- L-BFGS H_k g: one update + one apply, effective bandwidth of the paper
    if want("lbfgs"):
        lb = []
        gen = torch.Generator(device=dev).manual_seed(6)
        for n_l, m_l in ((1_000_000, 5), (1_000_000, 50), (10_000_000, 5), (10_000_000, 10),
                         (10_000_000, 50)):
            L = spx.lbfgs_create(n_l, m_l)
            dcurv = torch.rand(n_l, generator=gen, device=dev, dtype=torch.float64) * 1.5 + 0.5
            hist = []
            for _ in range(m_l + 4):
                s_ = torch.randn(n_l, generator=gen, device=dev, dtype=torch.float64)
                y_ = dcurv * s_ + 0.1 * torch.randn(n_l, generator=gen, device=dev, dtype=torch.float64)
                hist.append((s_, y_))
            g_ = torch.randn(n_l, generator=gen, device=dev, dtype=torch.float64)
            h0_ = torch.rand(n_l, generator=gen, device=dev, dtype=torch.float64) + 0.5
            p_ = torch.empty_like(g_)
            for s_, y_ in hist[:m_l]:
                L.update(s_, y_)
            evs = []
            for k in range(8):
                e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
                s_, y_ = hist[m_l + (k % 4)]
                e0.record()
                L.update(s_, y_)
                e1.record()
                L.apply(g_, h0_, p_)
                e2.record()
                evs.append((e0, e1, e2))
            torch.cuda.synchronize()
            # the same step through the fused entry point (S^T g in the update's pass)
            fevs = []
            for k in range(8):
                e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
                s_, y_ = hist[m_l + (k % 4)]
                e0.record()
                L.update_apply(s_, y_, g_, h0_, p_)
                e1.record()
                fevs.append((e0, e1))
            torch.cuda.synchronize()
            upd = statistics.median(a.elapsed_time(b) for a, b, _ in evs)
            app = statistics.median(b.elapsed_time(c) for _, b, c in evs)
            t_ms = statistics.median(a.elapsed_time(c) for a, _, c in evs)
            f_ms = statistics.median(a.elapsed_time(b) for a, b in fevs)
            be = 8 * n_l * (2 * m_l + 2) / (t_ms * 1e-3) / 1e9
            be_f = 8 * n_l * (2 * m_l + 2) / (f_ms * 1e-3) / 1e9
            y_passes = 1  # a with Y^T a (the update reads S only)
            col_bytes = 8 * n_l * m_l
            lb.append({"n": n_l, "m": m_l, "update_ms": round(upd, 4), "apply_ms": round(app, 4),
                       "total_ms": round(t_ms, 4), "effective_gbs": round(be, 1),
                       "hbm_bytes": col_bytes * (3 + y_passes) + 8 * 8 * n_l,
                       "hbm_gbs": round((col_bytes * (3 + y_passes) + 8 * 8 * n_l) / (t_ms * 1e-3) / 1e9, 1),
                       "fused_ms": round(f_ms, 4), "fused_effective_gbs": round(be_f, 1),
                       "fused_hbm_gbs": round((col_bytes * (2 + y_passes) + 8 * 8 * n_l) / (f_ms * 1e-3) / 1e9,
                                              1)})
            log(f"lbfgs n={n_l} m={m_l}: update {upd:.3f} ms apply {app:.3f} ms B_e {be:.0f} GB/s; "
                f"fused {f_ms:.3f} ms B_e {be_f:.0f} GB/s")
            L.destroy()
            del hist, dcurv, g_, h0_, p_
        out["lbfgs"] = {"points": lb,
                        "effective_bandwidth": "8 n (2m + 2) bytes / (T_update + T_apply): "
                                               "S and Y read once, g read, p written",
                        "hbm_bytes": "bytes this design moves: S read 3 times (update, S^T g, p), Y "
                                     "once (a with Y^T a), plus 8 vector passes; the fused step reads "
                                     "S twice",
                        "fused": "spx_lbfgs_update_apply: the same step with S^T g taken in the "
                                 "update's pass over S (bitwise the two calls)"}

    # ---- gradient on 256 x 256 elements
    if want("gradient256"):
        N = 256
        one = W.q1_poisson(N, 2, kappa=np.ones(N * N))
        w = one.dv_dlogk
        base = one.v - w
        _, theta, target, b = W.config5(N)
        G = spx.coo_preallocate(one.n, d(one.i), d(one.j))
        T = spx.coo_preallocate(one.n, d(target.i), d(target.j))
        T.set_values_coo(d(target.v))
        ustar = T.cg_solve(d(b), rtol=1e-12).x
        th = d(theta).requires_grad_(True)
        bd, based, wd = d(b), d(base), d(w)
        # one untimed forward and backward first: the first calls load kernel code
        u0 = AG.element_coefficient_solve(th, bd, G, based, wd, 16, rtol=1e-12)
        (0.5 * torch.sum((u0 - ustar) ** 2)).backward()
        th.grad = None
        fw_ms, u = timed(lambda: AG.element_coefficient_solve(th, bd, G, based, wd, 16, rtol=1e-12))
        loss = 0.5 * torch.sum((u - ustar) ** 2)
        bw_ms, _ = timed(lambda: loss.backward())
        out["gradient256"] = {"forward_ms": round(fw_ms, 2), "backward_ms": round(bw_ms, 2),
                              "loss": float(loss.detach())}
        log(f"gradient: forward {fw_ms:.2f} ms backward {bw_ms:.2f} ms")
    return out


def host_threads() -> int:
    """Host CPUs this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(grid: int, calls: int, full=None):
    """The oracle as it stands (plain C, gcc -O2) timed on the host, in two
    legs:

    * one thread on a bounded sample: its own COO assembly of the same 3-D
      Q1 workload at grid^3 elements, `calls` SpMV calls and 20 Jacobi-CG
      iterations;
    * every host thread (OpenMP rows and fixed dot blocks, bitwise the one-
      thread results) on the full-size matrix when `full` is given: its own
      assembly (one thread: the sort is sequential), `calls` SpMV calls,
      Jacobi-CG to 1e-10, and FP64 CG to 1e-12 on the log-normal values,
      whose solution is the reference for the GPU solutions' errors.

    `full` = (prob, b2, v3, b3, x_c3) with x_c3 the GPU's log-normal
    solutions by name.  Returns (baseline object, errors object or None)."""
    import numpy as np

    import oracle
    from paper_2406_08646_amd import workloads as W

    model, ncpu, nsock = host_cpu()
    threads = host_threads()
    oracle.set_threads(1)
    prob, x, _ = W.config2(grid)
    t0 = time.perf_counter()
    A = oracle.assemble(prob.n, prob.i, prob.j, prob.v)
    t_asm = time.perf_counter() - t0
    times = []
    for _ in range(calls):
        t0 = time.perf_counter()
        oracle.spmv(A, x)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    gbs = spmv_bytes(A.n, A.nnz) / med / 1e9
    t0 = time.perf_counter()
    oracle.coo_values(A.jmap, A.perm, prob.v)
    t_val = time.perf_counter() - t0
    b = np.random.default_rng(0).uniform(-1.0, 1.0, A.n)
    t0 = time.perf_counter()
    cg = oracle.pcg(A, b, 1e-30, maxit=20)
    t_cg = (time.perf_counter() - t0) / max(1, cg.iters)
    one = {
        "cores": 1, "value": round(gbs, 3), "unit": "GB/s",
        "sample": (f"{grid}^3-element 3-D Q1 matrix (n={A.n}, ncoo={prob.ncoo}, nnz={A.nnz})"),
        "assembly_s": round(t_asm, 3), "set_values_ms": round(t_val * 1e3, 2),
        "set_values_gbs": round(set_values_bytes(prob.ncoo, A.nvalid, A.nnz) / t_val / 1e9, 3),
        "spmv_ms": round(med * 1e3, 3), "cg_ms_per_iter": round(t_cg * 1e3, 3),
        "cg_gbs": round(cg_iteration_bytes(A.n, A.nnz) / t_cg / 1e9, 3),
    }
    del A, prob
    legs = [one]
    errors = None
    if full is not None:
        fprob, b2, v3, b3, x_c3 = full
        t0 = time.perf_counter()
        rowptr, col, jmap, perm = oracle.coo_pattern(fprob.n, fprob.i, fprob.j)
        t_pat = time.perf_counter() - t0
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        val2 = oracle.coo_values(jmap, perm, fprob.v)
        t_val2 = time.perf_counter() - t0
        F = oracle.CsrMatrix(fprob.n, rowptr, col, val2, jmap, perm, fprob.ncoo)
        xr = np.random.default_rng(0).uniform(-1.0, 1.0, F.n)
        times = []
        for _ in range(calls):
            t0 = time.perf_counter()
            oracle.spmv(F, xr)
            times.append(time.perf_counter() - t0)
        fmed = statistics.median(times)
        t0 = time.perf_counter()
        c2 = oracle.pcg(F, b2, 1e-10)
        t_c2 = time.perf_counter() - t0
        F3 = oracle.CsrMatrix(fprob.n, rowptr, col, oracle.coo_values(jmap, perm, v3), jmap, perm,
                              fprob.ncoo)
        del F, val2
        t0 = time.perf_counter()
        o64 = oracle.pcg(F3, b3, 1e-12)
        t_o64 = time.perf_counter() - t0
        nrm = float(np.linalg.norm(o64.x))
        bn = float(np.linalg.norm(b3))
        errors = {"reference": (f"oracle FP64 Jacobi-CG to 1e-12 on the log-normal matrix "
                                f"({o64.iters} iterations, relres {o64.relres:.3e})")}
        for name, xg in x_c3.items():
            errors[name] = {
                "rel_error": float(np.linalg.norm(xg - o64.x) / nrm),
                "true_relres": float(np.linalg.norm(b3 - oracle.spmv(F3, xg)) / bn)}
        legs.append({
            "cores": threads, "value": round(spmv_bytes(fprob.n, len(col)) / fmed / 1e9, 3),
            "unit": "GB/s",
            "sample": (f"timed {fprob.grid}^3-element 3-D Q1 matrix (n={fprob.n}, "
                       f"ncoo={fprob.ncoo}, nnz={len(col)})"),
            "symbolic_s_one_thread": round(t_pat, 2), "set_values_ms": round(t_val2 * 1e3, 1),
            "spmv_ms": round(fmed * 1e3, 3),
            "cg_1e-10_ms": round(t_c2 * 1e3, 1), "cg_1e-10_iters": c2.iters,
            "cg_ms_per_iter": round(t_c2 * 1e3 / max(1, c2.iters), 3),
            "lognormal_cg_1e-12_ms": round(t_o64 * 1e3, 1),
            "lognormal_cg_1e-12_iters": o64.iters,
        })
        oracle.set_threads(1)
    top = legs[-1]
    out = {
        "value": top["value"],
        "unit": "GB/s",
        "cores": top["cores"],
        "kind": "oracle",
        "sample": ("oracle SpMV GB/s (same byte count as the GPU figure) on the "
                   + top["sample"] + f" with {top['cores']} thread(s); legs: "
                   + "; ".join(f"{leg['cores']} thread(s) on the {leg['sample']}" for leg in legs)
                   + f"; host '{model}', {nsock} socket(s), {ncpu} logical CPUs, {threads} usable"),
        "legs": legs,
    }
    return out, errors


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=127, help="elements per side (127 = full size)")
    ap.add_argument("--spmv-calls", type=int, default=100)
    ap.add_argument("--check-every", type=int, default=20)
    ap.add_argument("--lanes", type=int, default=0, help="lanes per CSR row (0 = automatic)")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not bracket solver kernels with events (no roofline object)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-grid", type=int, default=63)
    ap.add_argument("--cpu-calls", type=int, default=10)
    ap.add_argument("--cpu-sample-only", action="store_true",
                    help="time the oracle on the small sample only (no full-size leg, no errors "
                         "against the FP64 oracle)")
    ap.add_argument("--extras", default=None,
                    help="comma-separated subset of the extra measurements to run (default: all): "
                         + ", ".join(EXTRAS))
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched / SpMM / gradient measurements")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a plain streaming kernel of known traffic (y = x + 1 over "
                         "2^27 doubles: 1 GiB read, 1 GiB written) for counter calibration")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path. "
              "Run with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2406_08646_amd import spx
    from paper_2406_08646_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    spx.load_library()
    torch.cuda.set_device(0)
    # the library's device memory comes from PyTorch's caching allocator, so
    # the symbolic stage's large temporaries are reused from step to step
    spx.use_torch_allocator(True)
    dev = torch.device("cuda", 0)
    N = args.grid

    if args.calibrate:
        ca = torch.ones(2**27, dtype=torch.float64, device=dev)
        cb = torch.empty_like(ca)
        for _ in range(3):
            torch.add(ca, 1.0, out=cb)
        torch.cuda.synchronize()
        del ca, cb
        log("calibration kernel done (3 x 1 GiB read + 1 GiB write)")

    log(f"generating the {N}^3-element workload")
    prob, x_np, b_np = W.config2(N)
    prob3, b3_np = W.config3(N)
    n, ncoo = prob.n, prob.ncoo
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    i_d, j_d = d(prob.i), d(prob.j)
    v2_d, v3_d = d(prob.v), d(prob3.v)
    x_d, b2_d, b3_d = d(x_np), d(b_np), d(b3_np)
    v3_np = prob3.v
    del prob3
    y_d = torch.empty_like(x_d)
    yt_d = torch.empty_like(x_d)
    torch.cuda.synchronize()
    log(f"inputs resident: n={n} ncoo={ncoo}")

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def run_step(profile: bool):
        rec = {}
        e = [ev() for _ in range(16)]  # e[0..11] used
        t0 = time.perf_counter()
        e[0].record()
        A = spx.coo_preallocate(n, i_d, j_d)
        e[1].record()
        A.set_values_coo(v2_d)
        e[2].record()
        if args.lanes:
            A.set_option(spx.OPT_SPMV_LANES, args.lanes)
        ms_mv, ms_mvt = [], []
        for _ in range(args.spmv_calls):
            s, t = ev(), ev()
            s.record()
            A.matmult(x_d, y_d)
            t.record()
            ms_mv.append((s, t))
        e[3].record()
        A.matmult_transpose(x_d, yt_d)  # builds the transpose
        e[4].record()
        for _ in range(args.spmv_calls):
            s, t = ev(), ev()
            s.record()
            A.matmult_transpose(x_d, yt_d)
            t.record()
            ms_mvt.append((s, t))
        e[5].record()
        r2 = A.cg_solve(b2_d, rtol=1e-10, check_every=args.check_every)
        e[6].record()
        # the same solve again with every kernel bracketed by events (the
        # roofline's launch times); the events slow the solve, so its wall
        # time is not the one reported
        A.set_option(spx.OPT_PROFILE, 1 if profile else 0)
        A.reset_profile()
        rp = A.cg_solve(b2_d, rtol=1e-10, check_every=args.check_every)
        prof = A.get_profile()
        A.set_option(spx.OPT_PROFILE, 0)
        e[10].record()
        A.set_values_coo(v3_d)
        e[7].record()
        r3 = A.cg_solve(b3_d, rtol=1e-10, check_every=args.check_every)
        e[8].record()
        rm = A.cg_solve_mixed(b3_d, rtol_outer=1e-10, rtol_inner=1e-4,
                              check_every=args.check_every, early_exit=False)
        e[9].record()
        re_ = A.cg_solve_mixed(b3_d, rtol_outer=1e-10, rtol_inner=1e-4,
                               check_every=args.check_every, early_exit=True)
        e[11].record()
        A.set_option(spx.OPT_IR_EARLY_EXIT, 0)
        nnz = A.nnz
        rec["walk"] = A.get_option(spx.OPT_SPMV_VARIANT)
        rec["window"] = A.get_window(arrays=False)
        A.destroy()
        torch.cuda.synchronize()
        rec["wall_ms"] = (time.perf_counter() - t0) * 1e3
        rec["preallocate_ms"] = e[0].elapsed_time(e[1])
        rec["set_values_ms"] = e[1].elapsed_time(e[2])
        rec["spmv_ms"] = [s.elapsed_time(t) for s, t in ms_mv]
        rec["spmvt_ms"] = [s.elapsed_time(t) for s, t in ms_mvt]
        rec["transpose_build_ms"] = e[3].elapsed_time(e[4])
        rec["cg64_ms"] = e[5].elapsed_time(e[6])
        rec["cg64"] = (r2.iters, r2.relres, r2.status)
        rec["cg64_profiled_ms"] = e[6].elapsed_time(e[10])
        rec["cg64_profiled_iters"] = rp.iters
        rec["set_values2_ms"] = e[10].elapsed_time(e[7])
        rec["cg64_ln_ms"] = e[7].elapsed_time(e[8])
        rec["cg64_ln"] = (r3.iters, r3.relres, r3.status)
        rec["mixed_ms"] = e[8].elapsed_time(e[9])
        rec["mixed"] = (rm.outer, rm.inner, rm.relres, rm.status)
        rec["mixed_early_ms"] = e[9].elapsed_time(e[11])
        rec["mixed_early"] = (re_.outer, re_.inner, re_.relres, re_.status)
        rec["x_c3"] = (r3.x, rm.x, re_.x)
        rec["profile"] = prof
        rec["nnz"] = nnz
        return rec

    profile = not args.no_profile
    for w in range(args.warmup):
        r = run_step(profile)
        log(f"warmup {w + 1}/{args.warmup}: {r['wall_ms']:.1f} ms")
    torch.cuda.synchronize()
    recs = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        r = run_step(profile)
        recs.append(r)
        log(f"step {k + 1}/{args.steps}: {r['wall_ms']:.1f} ms; cg {r['cg64'][0]} it; "
            f"lognormal fp64 {r['cg64_ln'][0]} it {r['cg64_ln_ms']:.1f} ms; mixed "
            f"{r['mixed'][0]} outer/{r['mixed'][1]} inner {r['mixed_ms']:.1f} ms; early exit "
            f"{r['mixed_early'][1]} inner {r['mixed_early_ms']:.1f} ms")
        if k + 1 < args.steps:
            r.pop("x_c3")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    # the last step's log-normal solutions, for their error against the FP64 oracle
    x_c3 = {name: t.cpu().numpy() for name, t in zip(("fp64", "mixed", "mixed_early_exit"),
                                                   recs[-1].pop("x_c3"))}

    nnz = recs[0]["nnz"]
    mv_bytes = spmv_bytes(n, nnz)
    walk = recs[0]["walk"]
    # bytes of the format the walk reads: 16-bit window columns for the
    # window walk; the staged x blocks are counted once in x (they come
    # through L2 for the neighbouring tiles)
    fmt_bytes = mv_bytes - 2 * nnz if walk == 4 else mv_bytes
    mv = [t for r in recs for t in r["spmv_ms"]]
    mvt = [t for r in recs for t in r["spmvt_ms"]]
    mv_med = statistics.median(mv)
    mvt_med = statistics.median(mvt)
    gbs = mv_bytes / (mv_med * 1e-3) / 1e9
    gbs_t = mv_bytes / (mvt_med * 1e-3) / 1e9
    med = lambda key: statistics.median(r[key] for r in recs)

    out = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_total * 1e3 / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"3-D Q1 trilinear Poisson, {N}^3 elements ({N + 1}^3 nodes), "
                         f"{ncoo} FP64 COO triplets -> {nnz} CSR nnz (27-point rows); "
                         f"{args.spmv_calls} MatMult + {args.spmv_calls} MatMultTranspose; "
                         "Jacobi-CG to 1e-10; log-normal (sigma=1) values: FP64 CG vs "
                         "FP32/FP64 refinement to 1e-10"),
            "n": n, "ncoo": ncoo, "nnz": nnz,
        },
        "spmv": {
            "median_ms": round(mv_med, 4), "mean_ms": round(statistics.fmean(mv), 4),
            "bytes_per_call": mv_bytes, "pct_of_peak": round(100 * gbs / PEAK_HBM_GBS, 2),
            "walk": WALKS.get(walk, str(walk)), "format_bytes_per_call": fmt_bytes,
            "format_gbs": round(fmt_bytes / (mv_med * 1e-3) / 1e9, 1),
            "window": recs[0]["window"],
            "transpose_median_ms": round(mvt_med, 4), "transpose_gbs": round(gbs_t, 2),
            "transpose_build_ms": round(med("transpose_build_ms"), 3),
        },
        "assembly": {
            "preallocate_ms": round(med("preallocate_ms"), 3),
            "preallocate_bytes": preallocate_bytes(n, ncoo, ncoo, nnz),
            "preallocate_gbs": round(preallocate_bytes(n, ncoo, ncoo, nnz)
                                     / (med("preallocate_ms") * 1e-3) / 1e9, 1),
            "preallocate_frac": round(preallocate_bytes(n, ncoo, ncoo, nnz)
                                      / (med("preallocate_ms") * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "preallocate_design_bytes": preallocate_design_bytes(n, ncoo, nnz),
            "set_values_ms": round(med("set_values_ms"), 4),
            "set_values_gbs": round(set_values_bytes(ncoo, ncoo, nnz)
                                    / (med("set_values_ms") * 1e-3) / 1e9, 1),
            "set_values_bytes": set_values_bytes(ncoo, ncoo, nnz),
        },
    }
    if profile:
        tot_ms = sum(r["profile"]["spmv_dot_f64"][0] for r in recs)
        cnt = sum(r["profile"]["spmv_dot_f64"][1] for r in recs)
        avg_ms = tot_ms / max(1, cnt)
        ach = mv_bytes / (avg_ms * 1e-3) / 1e9
        out["roofline"] = {
            "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": measured_traffic(),
            "kernel": (f"k_cg_spmv ({WALKS.get(walk, walk)} walk: q = A p with the p.q partial, "
                       "FP64)"),
            "bytes_per_launch": mv_bytes, "format_bytes_per_launch": fmt_bytes,
            # the same launches counted in the bytes of the format the walk
            # reads (16-bit window columns): the stricter figure
            "format_achieved": round(fmt_bytes / (avg_ms * 1e-3) / 1e9, 1),
            "format_frac": round(fmt_bytes / (avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "avg_launch_ms": round(avg_ms, 4), "launches": cnt,
            "source_hash": kernel_source_hash(),
        }
        out["solver_kernels_ms"] = {k: [round(sum(r["profile"][k][0] for r in recs) /
                                               max(1, sum(r["profile"][k][1] for r in recs)), 4),
                                        sum(r["profile"][k][1] for r in recs)]
                                    for k in spx.PROFILE_KINDS[:3]}
    if not args.no_extras:
        only = None
        if args.extras:
            only = set(args.extras.split(","))
            unknown = only - set(EXTRAS)
            if unknown:
                print(f"bench.py: unknown extras {sorted(unknown)}; choose from {', '.join(EXTRAS)}",
                      file=sys.stderr)
                return 2
        out["extras"] = run_extras(spx, W, torch, np, dev, prob, x_np, b_np, log, only)
    errors = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on the {args.cpu_grid}^3-element sample (1 thread) and the "
            f"full-size matrix ({host_threads()} threads)")
        full = None if args.cpu_sample_only else (prob, b_np, v3_np, b3_np, x_c3)
        out["cpu_baseline"], errors = cpu_baseline(args.cpu_grid, args.cpu_calls, full)
    # the whole CG half of the metric, last on the line
    first = recs[0]
    out["cg"] = {
        "kappa1_fp64": {"ms": round(med("cg64_ms"), 2), "iters": first["cg64"][0],
                        "relres": first["cg64"][1], "status": first["cg64"][2],
                        "ms_per_iter": round(med("cg64_ms") / max(1, first["cg64"][0]), 4),
                        "profiled_ms": round(med("cg64_profiled_ms"), 2),
                        "gbs_per_iter": round(cg_iteration_bytes(n, nnz) * first["cg64"][0]
                                              / (med("cg64_ms") * 1e-3) / 1e9, 1)},
        "lognormal_fp64": {"ms": round(med("cg64_ln_ms"), 2), "iters": first["cg64_ln"][0],
                           "relres": first["cg64_ln"][1], "status": first["cg64_ln"][2]},
        "lognormal_mixed": {"inner_rule": "rtol_inner 1e-4 (literal)",
                            "ms": round(med("mixed_ms"), 2), "outer": first["mixed"][0],
                            "inner": first["mixed"][1], "relres": first["mixed"][2],
                            "status": first["mixed"][3]},
        "lognormal_mixed_early_exit": {"inner_rule": "max(rtol_inner ||r32||, rtol_outer ||b|| / 2)",
                                       "ms": round(med("mixed_early_ms"), 2),
                                       "outer": first["mixed_early"][0],
                                       "inner": first["mixed_early"][1],
                                       "relres": first["mixed_early"][2],
                                       "status": first["mixed_early"][3]},
        "mixed_speedup": round(med("cg64_ln_ms") / med("mixed_ms"), 3),
        "mixed_speedup_early_exit": round(med("cg64_ln_ms") / med("mixed_early_ms"), 3),
        "error_vs_oracle64": errors,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
