#!/usr/bin/env python
"""Benchmark of the vertex-model hot path on one MI355X.

Headline workload (the force-kernel throughput case): one periodic Voronoi
tissue of 10^6 cells (uniform-random seeds, box side 1000; 2e6 3-valent
vertices, 3e6 edges), FP32 positions, K_A = A0 = K_P = 1, P0 = 3.75,
per-edge lambda ~ U[0.05, 0.15], fixed topology.  One step is one energy +
force evaluation (the fused tile kernel, which forms the cell coefficients
in LDS and the forces from them, then a one-block finish of the
deterministic FP64 energy and max-force sums), replayed from captured
graphs with the inputs resident in HBM; exactly --warmup untimed and
--steps timed evaluations.  The timed region is bracketed by HIP events on
the launch stream, after a synchronisation and a ~1.5 ms device-side delay
that covers the host's submission of the first timed graph launch.

Printed: one JSON line with the whole-job vertex-force evaluations per
second; the roofline of the dominant kernel (the fused evaluation kernel,
timed alone with HIP events on the stream it is launched on) against the
algorithmic floor of an evaluation, 34 bytes per vertex (positions in,
forces out, one 3-neighbour list, each edge tension once), warm (working set
served partly from the 256 MB Infinity Cache) and cold (after a 512 MiB
write), with the two-pass kernels (cell pass, vertex pass) timed the same
way for reference; the oracle timed on
the host cores (one thread and all cores of the box's share); and, unless
--no-secondary, the other workloads: the 100-cell and 10^4-cell single
relaxations, the 512-tissue batched relaxation and the 64-tissue batched
hypergradients.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "vertex-force evals/s; param-gradients/s (batched adjoint vs plain) at 1e-6 tol"
FLOOR_B_PER_VERTEX = 34   # positions in 8 + forces out 8 + 3-neighbour list 12 + lambda 6
SLEEP_CYCLES = 240000     # device-side delay before the timed region (~1.5 ms on MI355X)
COUNTERS = os.path.join(ROOT, "profiles", "eval_fused_1m_cells_counters.txt")
SQ_COUNTERS = os.path.join(ROOT, "profiles", "eval_fused_1m_cells_sq_counters.txt")
SIMDS, CLOCK_HZ, VALU_CYCLES = 1024, 2.4e9, 4   # 256 CUs x 4 SIMDs; a wave64 VALU op: 4 cycles


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def fused_design_bytes(n_vert, n_edge, ts):
    """Bytes the fused evaluation kernel must move at least once (FP32), from
    the tile tables' layout `ts` (Tissue.tile_stats())."""
    return (ts["tiles"] * 16                 # per-tile counts
            + ts["cells"] * 4                # tile cell lists
            + ts["halo"] * (4 + 8)           # halo ids and their positions
            + (ts["cells"] + ts["tiles"]) * 2  # row starts
            + ts["corners"] * 2              # corner references
            + n_vert * (16 + 8)              # local star + edge ids
            + n_vert * 8                     # own position
            + n_edge * 4                     # lambda of every edge
            + n_vert * 8)                    # forces written


def design_bytes(n_vert, n_cell, n_edge, n_he):
    """Bytes each pass of the two-pass layout must move at least once (FP32)."""
    vertex = (n_vert * 8          # own position
              + n_vert * 36       # star: 3 neighbour ids, 3 cell ids, 3 edge ids
              + n_cell * 8        # (cA, cP) of every cell
              + n_edge * 4        # lambda of every edge
              + n_vert * 8)       # forces written
    cell = ((n_cell + 1) * 4      # row offsets
            + n_cell * 4          # side counts
            + n_he * 4            # corner ids
            + n_vert * 8          # positions
            + n_cell * 8)         # (cA, cP) written
    return vertex, cell


KERNEL_SOURCES = ["include/vtx.h", "paper_2604_06896_amd/csrc/vtx_kernels.hip",
                  "paper_2604_06896_amd/csrc/vtx_device.h",
                  "paper_2604_06896_amd/csrc/vtx_internal.h",
                  "paper_2604_06896_amd/csrc/vtx_launch.h"]


def kernel_source_sha():
    """Hash of the sources the evaluation kernels are compiled from, to tell
    whether committed counters still describe the kernels that run."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def read_summary(path, sha, key):
    """A figure `key: value` from a committed counter summary, or None if the
    summary is missing or was taken on other kernel sources."""
    vals = {}
    try:
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith(("#", "|", " ")):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
    except OSError:
        return None
    if vals.get("kernel_source_sha") != sha:
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def read_traffic(path, sha):
    """HBM bytes per fused-evaluation launch from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel
    calibration), or None if the summary is missing or was taken on other
    kernel sources."""
    if not os.path.exists(path):
        return None, "no counter summary"
    v = read_summary(path, sha, "fused_eval_bytes_per_launch")
    if v is None:
        return None, "counters taken on other kernel sources, or no fused-evaluation figure"
    return v, "rocprofv3 FETCH_SIZE + WRITE_SIZE"


# --------------------------------------------------------------- CPU baseline
# The oracle (plain FP64 C, one thread per process) on the machine's host cores.
# Each worker is a fresh process that loads the inputs from .npy files.

def _worker(job):
    import numpy as np
    sys.path.insert(0, ROOT)
    import oracle as O
    kind, d, arg = job

    def load(name):
        return np.load(os.path.join(d, name + ".npy"))

    def params(prefix):
        from types import SimpleNamespace
        return SimpleNamespace(KA=load(prefix + "KA"), A0=load(prefix + "A0"), KP=load(prefix + "KP"),
                               P0=load(prefix + "P0"), lam=load(prefix + "lam"))

    if kind == "eval":          # energy + forces, repeated for `arg` seconds
        m = O.Mesh(load("c3_he"), int(load("c3_nv")), float(load("c3_L")), float(load("c3_L")))
        X, p = load("c3_X"), params("c3_")
        n, t0 = 0, time.perf_counter()
        while True:
            O.energy_forces(m, X, p)
            n += 1
            if time.perf_counter() - t0 > arg:
                break
        return n, time.perf_counter() - t0
    if kind == "relax":         # a fixed number of relaxation steps
        pre, opts = arg
        m = O.Mesh(load(pre + "he"), int(load(pre + "nv")), float(load(pre + "L")),
                   float(load(pre + "L")))
        X = load(pre + "X").copy()
        t0 = time.perf_counter()
        r = O.relax(m, X, params(pre), patience=1, **opts)
        return r, time.perf_counter() - t0
    if kind == "adjoint":       # one adjoint hypergradient (CG to 1e-8)
        m = O.Mesh(load("c5_he"), int(load("c5_nv")), float(load("c5_L")), float(load("c5_L")))
        X, p, b = load("c5_X"), params("c5_"), load("c5_b")
        t0 = time.perf_counter()
        _, info = O.adjoint_grad(m, X, p, b, tol=1e-8)
        return info, time.perf_counter() - t0
    raise ValueError(kind)


def _host():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"nproc": os.cpu_count(), "affinity_cpus": aff, "cpu_model": model}


def cpu_baseline(t, X32, lam32, args, secondary_inputs):
    """The oracle, untuned, on the machine's host cores: one thread and one
    process per core of the box's share (at most 16), each process running
    the plain single-threaded oracle on its own copy of the inputs."""
    import multiprocessing as mp

    import numpy as np

    from paper_2604_06896_amd import tissue_gen as g
    host = _host()
    P = max(1, min(16, host["affinity_cpus"] or 1))
    d = tempfile.mkdtemp(prefix="vtx_bench_", dir="/tmp")

    def save(name, a):
        np.save(os.path.join(d, name + ".npy"), np.asarray(a))

    def save_params(pre, p, nc, ne):
        for k in ("KA", "A0", "KP", "P0"):
            save(pre + k, np.broadcast_to(getattr(p, k), (nc,)).astype(np.float64))
        save(pre + "lam", np.broadcast_to(p.lam, (ne,)).astype(np.float64))

    # config 3: the headline tissue, FP64 upcast of the FP32 inputs
    save("c3_he", t.he)
    save("c3_nv", t.n_vert)
    save("c3_L", t.Lx)
    save("c3_X", X32.astype(np.float64))
    p3 = g.uniform_params(t, P0=3.75)
    p3.lam = lam32.astype(np.float64)
    save_params("c3_", p3, t.n_cell, t.n_edge)
    for pre, (tt, pp, _) in secondary_inputs.items():
        save(pre + "he", tt.he)
        save(pre + "nv", tt.n_vert)
        save(pre + "L", tt.Lx)
        save(pre + "X", tt.X)
        save_params(pre, pp, tt.n_cell, tt.n_edge)
    ctx = mp.get_context("spawn")
    out = {"kind": "oracle", "host": host}
    with ctx.Pool(P) as pool:
        s = args.cpu_seconds
        n1, dt1 = pool.apply(_worker, (("eval", d, s),))
        one = t.n_vert * n1 / dt1
        res = pool.map(_worker, [("eval", d, s)] * P)
        allc = sum(t.n_vert * n / dt for n, dt in res)
        log(f"oracle, 1e6 cells: {one:.3e} vertex-force evals/s on one thread, {allc:.3e} on {P}")
        out.update({"value": allc, "unit": "vertex-force evals/s", "cores": P,
                    "single_thread": one,
                    "sample": f"FP64 energy+force evaluations of the same 1e6-cell tissue for "
                              f"{s:.0f} s: {n1} on one thread, {sum(n for n, _ in res)} in "
                              f"{P} processes (one per core)"})
        if "c1_" in secondary_inputs:
            (r, dt), (r2, dt2) = pool.map(_worker, [
                ("relax", d, ("c1_", dict(eta=1e-2, tol=1e-6, max_iter=200000, t1_enable=True,
                                           l_min=0.01))),
                ("relax", d, ("c1_", dict(eta=1e-2, tol=1e-6, max_iter=20000,
                                           t1_enable=False)))])
            out["config1"] = {"with_t1": {"iters": r["iters"], "n_t1": r["n_t1"],
                                          "status": r["status"], "s": dt},
                              "without_t1_20000_steps": {"status": r2["status"],
                                                         "max_f": r2["max_f"], "s": dt2}}
            log(f"oracle, 100 cells: relaxation with T1 {r['iters']} steps in {dt:.2f}s")
        if "c2_" in secondary_inputs:
            n2 = secondary_inputs["c2_"][2]
            r, dt = pool.apply(_worker, (("relax", d, ("c2_", dict(
                eta=3e-3, tol=0.0, max_iter=n2, t1_enable=True, l_min=0.01))),))
            out["config2"] = {"steps": n2, "s": dt, "ms_per_step": dt / n2 * 1e3}
            log(f"oracle, 1e4 cells: {n2} relaxation steps with T1 in {dt:.2f}s")
        c4 = sorted(k for k in secondary_inputs if k.startswith("c4_"))
        if c4:
            n4 = secondary_inputs[c4[0]][2]
            res = pool.map(_worker, [("relax", d, (k, dict(eta=3e-3, tol=0.0, max_iter=n4,
                                                           t1_enable=True, l_min=0.01)))
                                     for k in c4])
            vi = [secondary_inputs[k][0].n_vert * n4 / dt for k, (_, dt) in zip(c4, res)]
            out["config4"] = {"tissues_sampled": len(c4), "steps_each": n4,
                              "cells": [secondary_inputs[k][0].n_cell for k in c4],
                              "vertex_iters_per_s_single_thread_median": float(np.median(vi)),
                              "vertex_iters_per_s_all_cores": float(sum(vi)), "cores": len(c4)}
            log(f"oracle, 512-tissue workload sample: {sum(vi):.3e} vertex-iterations/s on "
                f"{len(c4)} cores")
        if args.c5_fixture:
            import sys as _s
            _s.path.insert(0, os.path.join(ROOT, "tests", "golden"))
            import make_inverse_equilibrium as mk
            t5, X5, p5 = mk.load()
            rng = np.random.default_rng(7)
            Xt5 = X5 + rng.normal(0, 0.05, X5.shape)
            save("c5_he", t5.he)
            save("c5_nv", t5.n_vert)
            save("c5_L", t5.Lx)
            save("c5_X", X5)
            save("c5_b", (X5 - Xt5) / t5.n_vert)
            save_params("c5_", p5, t5.n_cell, t5.n_edge)
            res = pool.map(_worker, [("adjoint", d, None)] * P)
            per = [dt for _, dt in res]
            out["config5"] = {"adjoint_s_single_thread_median": float(np.median(per)),
                              "cg_iters": int(res[0][0]["iters"]),
                              "grads_per_s_all_cores": float(sum(1.0 / x for x in per)),
                              "cores": P,
                              "sample": "oracle adjoint (CG to 1e-8, FP64) of the first "
                                        "1000-cell inverse-workload tissue at its oracle "
                                        "equilibrium, v2v cost to a perturbed target, one "
                                        "gradient per process"}
            log(f"oracle adjoint, 1000 cells: {np.median(per):.2f} s per gradient on one thread")
    for f in os.listdir(d):
        os.remove(os.path.join(d, f))
    os.rmdir(d)
    return out


# ---------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--graph-evals", type=int, default=50, help="evaluations per captured graph")
    ap.add_argument("--kernel-reps", type=int, default=500)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-cell", type=int, default=1000000)
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the other workloads (single relaxations, batched relaxation, "
                         "hypergradients)")
    ap.add_argument("--batch-tissues", type=int, default=512)
    ap.add_argument("--batch-max-iter", type=int, default=200000)
    ap.add_argument("--grad-tissues", type=int, default=64)
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--cold-reps", type=int, default=50,
                    help="evaluations timed one by one after a 512 MiB cache flush")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (known bytes) to calibrate "
                         "hardware traffic counters")
    args = ap.parse_args()
    args.c5_fixture = os.path.exists(os.path.join(ROOT, "tests", "golden",
                                                  "inverse_tissue0_equilibrium.txt"))

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library "
              "runs on a single MI355X and has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2604_06896_amd import tissue_gen as g
    from paper_2604_06896_amd import vtx as V

    V.lib()  # fails loudly if the HIP library is missing
    t0 = time.time()
    t, p = g.workload_force_1m(n_cell=args.n_cell)
    log(f"generated {t.n_cell} cells / {t.n_vert} vertices in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    T = V.Tissue.from_tissue(t)
    X = torch.as_tensor(t.X, dtype=torch.float32, device=dev)
    lam = torch.as_tensor(p.lam, dtype=torch.float32, device=dev)
    P = V.Params(KA=1.0, A0=1.0, KP=1.0, P0=3.75, lam=lam)
    cp, keep = P.to_c(torch.float32, dev)
    E = torch.empty((), dtype=torch.float64, device=dev)
    F = torch.empty_like(X)
    mf = torch.empty((), dtype=torch.float64, device=dev)

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 10 x 268435456-byte device copies")
        del src, dst

    def one_eval():
        T.energy_forces_into(X, cp, E, F, mf, mode="f32")

    def capture(fn, n):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            for _ in range(n):
                fn()
        return gr

    # eager warm-up of the library (not counted), then graphs of G
    # evaluations and of the remainders, so that exactly --warmup and
    # --steps evaluations run
    for _ in range(3):
        one_eval()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        one_eval()
    torch.cuda.current_stream().wait_stream(s)
    G = max(1, args.graph_evals)
    graphs = {G: capture(one_eval, G)}

    def run_evals(n):
        for _ in range(n // G):
            graphs[G].replay()
        r = n % G
        if r:
            if r not in graphs:
                graphs[r] = capture(one_eval, r)
            graphs[r].replay()

    run_evals(args.steps % G or G)       # capture the remainder graph before timing
    torch.cuda.synchronize()
    run_evals(args.warmup)
    torch.cuda.synchronize()
    # check a replayed evaluation against an eager one
    E_g, F_g = E.clone(), F.clone()
    one_eval()
    torch.cuda.synchronize()
    assert torch.equal(F_g, F) and E_g.item() == E.item(), "graph replay differs from eager"

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    # A short device-side delay (~1.5 ms) ahead of the start event: the host
    # submits the graph launches while it runs, so the events bracket the
    # GPU's execution of exactly --steps evaluations and not the host's
    # launch latency of an idle GPU (about 48 us once, which would add
    # 2.4 us per evaluation to a 20-step run).  The host-inclusive wall time
    # from the synchronisation on is logged beside it.
    w0 = time.perf_counter()
    torch.cuda._sleep(SLEEP_CYCLES)
    ev0.record()
    run_evals(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    steps = args.steps
    value = t.n_vert * steps / (ms / 1e3)
    log(f"{steps} evaluations in {ms:.3f} ms (host wall from the synchronisation, including "
        f"the ~1.5 ms delay and the launch: {wall * 1e3:.2f} ms): "
        f"{ms / steps * 1e3:.2f} us/eval, E = {E.item():.6f}, max|F| = {mf.item():.4f}")

    # ---- dominant kernel alone: the fused evaluation (forces only: no
    # energy or max-force sums, hence no finish launch), then the two-pass
    # kernels for reference; HIP events on the stream they are launched on
    # (torch's current stream)
    coeffs = T.cell_coeffs(X, P, mode="f32")
    R = max(G, (args.kernel_reps // G) * G)

    def timed_graph(fn):
        gr = capture(fn, G)
        gr.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(R // G):
            gr.replay()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / R

    F2 = torch.empty_like(X)
    fused = lambda: T.energy_forces_into(X, cp, None, F2, None, mode="f32")  # noqa: E731
    f_ms = timed_graph(fused)
    v_ms = timed_graph(lambda: T.vertex_forces_into(X, cp, coeffs, F2, mode="f32"))
    c_ms = timed_graph(lambda: V.lib().vtx_cell_coeffs(T.handle, V.F32, V._ptr(X), V.C.byref(cp),
                                                       V._ptr(coeffs), V._stream()))
    ts = T.tile_stats()
    fb = fused_design_bytes(t.n_vert, t.n_edge, ts)
    vb, cb = design_bytes(t.n_vert, t.n_cell, t.n_edge, t.n_he)
    floor = FLOOR_B_PER_VERTEX * t.n_vert
    log(f"fused evaluation kernel {f_ms * 1e3:.2f} us ({floor / f_ms / 1e6:.0f} GB/s of the "
        f"34 B/vertex floor, {fb / f_ms / 1e6:.0f} GB/s of its design bytes, "
        f"{fb / t.n_vert:.1f} B/vertex; tiles {ts})")
    log(f"two-pass reference: vertex pass {v_ms * 1e3:.2f} us, cell pass {c_ms * 1e3:.2f} us")
    sha = kernel_source_sha()
    traffic, traffic_src = read_traffic(COUNTERS, sha)

    # ---- cold caches: 512 MiB written between evaluations (not timed), so
    # that nothing of the ~150 MB an evaluation touches is left in the
    # 256 MB Infinity Cache or the L2s
    g1 = capture(one_eval, 1)
    gf1 = capture(fused, 1)
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)

    def cold(gr, n):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(n)]
        for i, (a, b) in enumerate(evs):
            flush.fill_(i & 255)
            a.record()
            gr.replay()
            b.record()
        torch.cuda.synchronize()
        return sorted(a.elapsed_time(b) for a, b in evs)[n // 2]  # median, ms

    cold_eval_ms = cold(g1, args.cold_reps)
    cold_f_ms = cold(gf1, args.cold_reps)
    del flush, g1, gf1
    log(f"cold caches: evaluation {cold_eval_ms * 1e3:.2f} us, fused kernel {cold_f_ms * 1e3:.2f} "
        f"us ({floor / cold_f_ms / 1e6:.0f} GB/s of the floor)")

    roofline = {
        "bound": "hbm", "kernel": "k_eval_fused (the whole evaluation: cell coefficients in "
                                  "LDS, then forces)",
        "achieved": floor / f_ms / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": floor / f_ms / 1e6 / HBM_PEAK_GBS, "traffic": traffic,
        "bytes_per_launch": floor,
        "bytes_basis": "algorithmic floor of an evaluation, 34 B per vertex: positions in 8, "
                       "forces out 8, one 3-neighbour list 12, each edge tension once 6",
        "us_per_launch": f_ms * 1e3,
        "timing": "warm: launches back to back, the working set partly served from the 256 MB "
                  "Infinity Cache; forces only (the energy and max-force sums add a one-block "
                  "finish launch, included in ms_per_step)",
        "traffic_source": traffic_src,
        "traffic_over_floor": traffic / floor if traffic else None,
        "design": {"bytes_per_launch": fb, "bytes_per_vertex": fb / t.n_vert,
                   "achieved": fb / f_ms / 1e6, "frac": fb / f_ms / 1e6 / HBM_PEAK_GBS,
                   "basis": "the tile tables' bytes, each array once", "tile_stats": ts},
        "cold_caches": {"fused_kernel_us": cold_f_ms * 1e3,
                        "achieved": floor / cold_f_ms / 1e6,
                        "frac": floor / cold_f_ms / 1e6 / HBM_PEAK_GBS,
                        "design_frac": fb / cold_f_ms / 1e6 / HBM_PEAK_GBS,
                        "evaluation_us": cold_eval_ms * 1e3},
        "two_pass_reference": {
            "vertex_pass_us": v_ms * 1e3, "vertex_pass_design_bytes": vb,
            "cell_pass_us": c_ms * 1e3, "cell_pass_design_bytes": cb,
            "vertex_pass_floor_frac": floor / v_ms / 1e6 / HBM_PEAK_GBS},
        "kernel_source_sha": sha,
    }
    valu = read_summary(SQ_COUNTERS, sha, "valu_wave_instructions_per_launch")
    roofline["alu"] = None if valu is None else {
        "valu_wave_instructions": valu,
        "issue_frac": valu * VALU_CYCLES / (SIMDS * CLOCK_HZ * f_ms / 1e3),
        "basis": "SQ_INSTS_VALU of the committed counter summary (median over the kernel's "
                 "dispatches with and without the energy sums) x 4 cycles per wave64 VALU "
                 "instruction, over the 1024 SIMDs at 2.4 GHz for the fused kernel's "
                 "measured time"}
    del F2, coeffs
    torch.cuda.empty_cache()

    # ---- secondary workloads (GPU), then the oracle on the host cores
    secondary = None
    sec_inputs = {}
    if not args.no_secondary:
        from paper_2604_06896_amd import suite
        secondary = {}
        w0 = time.perf_counter()
        secondary["single_100_cells"] = suite.single_100(log=log)
        c2 = suite.single_10k(log=log)
        secondary["single_10k_cells"] = c2
        secondary["batched_relax"] = suite.batched_relax(
            n_tissue=args.batch_tissues, max_iter=args.batch_max_iter,
            plain_sample=args.plain_sample, block_threads=1024, log=log)
        secondary["param_gradients"] = suite.param_gradients(
            n_tissue=args.grad_tissues, plain_sample=min(args.plain_sample, 8), log=log)
        log(f"secondary measurements took {time.perf_counter() - w0:.1f}s")
        t1w, p1w = g.workload_single_100()
        sec_inputs["c1_"] = (t1w, p1w, None)
        t2w, p2w = g.workload_single_10k()
        sec_inputs["c2_"] = (t2w, p2w, 50)
        for k, (tk, pk) in enumerate(suite.batch_sample(16)):
            sec_inputs[f"c4_{k:02d}_"] = (tk, pk, 500)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(t, X.cpu().numpy(), lam.cpu().numpy(), args, sec_inputs)
        if secondary and "config2" in cpu:
            c2 = secondary["single_10k_cells"]
            cpu["config2"]["extrapolated_s_to_gpu_step_count"] = \
                cpu["config2"]["ms_per_step"] * c2["iters"] / 1e3

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "vertex-force evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "force-kernel throughput: periodic Voronoi tissue of 1e6 cells "
                               "(box 1000), FP32 positions, fixed topology, one energy+force "
                               "evaluation per step",
                   "n_cell": t.n_cell, "n_vert": t.n_vert, "n_edge": t.n_edge,
                   "graph_evals": G},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
