#!/usr/bin/env python
"""Benchmark of the vertex-model hot path on one MI355X.

Workload (the force-kernel throughput case): one periodic Voronoi tissue of
10^6 cells (uniform-random seeds, box side 1000; 2e6 3-valent vertices, 3e6
edges), FP32 positions, K_A = A0 = K_P = 1, P0 = 3.75, per-edge lambda ~
U[0.05, 0.15], fixed topology.  One step is one energy + force evaluation
(cell pass + vertex pass + deterministic FP64 energy/max-force reductions);
steps are replayed from a captured graph, inputs resident in HBM.

Printed: one JSON line with the whole-job vertex-force evaluations per
second, the roofline of the dominant kernel (the vertex pass, timed alone
with HIP events on the stream it is launched on; also with cold caches,
after a 512 MiB write evicts the Infinity Cache), the oracle timed on the
host cores as a CPU baseline, and (unless --no-secondary) the batched
relaxation and hypergradient measurements.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "vertex-force evals/s; param-gradients/s (batched adjoint vs plain) at 1e-6 tol"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(n_vert, n_cell, n_edge, n_he):
    """Bytes each pass must move at least once (FP32 layout, ideal reuse)."""
    vertex = (n_vert * 8          # own position
              + n_vert * 36       # star: 3 neighbour ids, 3 cell ids, 3 edge ids
              + n_cell * 8        # (cA, cP) of every cell
              + n_edge * 4        # lambda of every edge
              + n_vert * 8)       # forces written
    cell = ((n_cell + 1) * 4      # row offsets
            + n_he * 4            # corner ids
            + n_vert * 8          # positions
            + n_cell * 8)         # (cA, cP) written
    return vertex, cell


def read_traffic(path):
    """HBM bytes per launch of the vertex pass from a committed counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB, scaled by the copy-kernel
    calibration), or None."""
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("vertex_pass_bytes_per_launch:"):
                    return float(line.split(":")[1])
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--graph-evals", type=int, default=50, help="evaluations per captured graph")
    ap.add_argument("--kernel-reps", type=int, default=500)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-cell", type=int, default=1000000)
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the batched relaxation and hypergradient measurements")
    ap.add_argument("--batch-tissues", type=int, default=512)
    ap.add_argument("--batch-max-iter", type=int, default=200000)
    ap.add_argument("--grad-tissues", type=int, default=64)
    ap.add_argument("--plain-sample", type=int, default=2)
    ap.add_argument("--cold-reps", type=int, default=50,
                    help="evaluations timed one by one after a 512 MiB cache flush")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (known bytes) to calibrate "
                         "hardware traffic counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library "
              "runs on a single MI355X and has no multi-GPU path)", file=sys.stderr)
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

    G = max(1, min(args.graph_evals, args.steps))
    steps = (args.steps // G) * G
    warm = max(G, (args.warmup // G) * G)

    def one_eval():
        T.energy_forces_into(X, cp, E, F, mf, mode="f32")

    # eager warm-up, then capture G evaluations in one graph
    for _ in range(3):
        one_eval()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        one_eval()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(G):
            one_eval()
    for _ in range(warm // G):
        graph.replay()
    torch.cuda.synchronize()
    # check the replayed evaluation against an eager one
    E_g, F_g = E.clone(), F.clone()
    one_eval()
    torch.cuda.synchronize()
    assert torch.equal(F_g, F) and E_g.item() == E.item(), "graph replay differs from eager"

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(steps // G):
        graph.replay()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    value = t.n_vert * steps / (ms / 1e3)
    log(f"{steps} evaluations in {ms:.2f} ms (wall {wall * 1e3:.2f} ms): "
        f"{ms / steps * 1e3:.2f} us/eval, E = {E.item():.6f}, max|F| = {mf.item():.4f}")

    # ---- dominant kernel alone: vertex pass (and cell pass), HIP events on
    # the stream they are launched on (torch's current stream)
    coeffs = T.cell_coeffs(X, P, mode="f32")
    R = max(G, (args.kernel_reps // G) * G)

    def timed_graph(fn):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            for _ in range(G):
                fn()
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
    v_ms = timed_graph(lambda: T.vertex_forces_into(X, cp, coeffs, F2, mode="f32"))
    c_ms = timed_graph(lambda: V.lib().vtx_cell_coeffs(T.handle, V.F32, V._ptr(X), V.C.byref(cp),
                                                       V._ptr(coeffs), V._stream()))
    vb, cb = algorithmic_bytes(t.n_vert, t.n_cell, t.n_edge, t.n_he)
    v_gbs = vb / (v_ms / 1e3) / 1e9
    c_gbs = cb / (c_ms / 1e3) / 1e9
    log(f"vertex pass {v_ms * 1e3:.2f} us ({v_gbs:.0f} GB/s algorithmic), "
        f"cell pass {c_ms * 1e3:.2f} us ({c_gbs:.0f} GB/s)")
    traffic = read_traffic(os.path.join(ROOT, "profiles", "vertex_pass_1m_cells_counters.txt"))

    # ---- cold caches: 512 MiB written between evaluations (not timed), so
    # that nothing of the ~180 MB an evaluation touches is left in the
    # 256 MB Infinity Cache or the L2s
    g1 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g1):
        one_eval()
    gv1 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gv1):
        T.vertex_forces_into(X, cp, coeffs, F2, mode="f32")
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
    cold_v_ms = cold(gv1, args.cold_reps)
    del flush, g1, gv1
    log(f"cold caches: evaluation {cold_eval_ms * 1e3:.2f} us, vertex pass {cold_v_ms * 1e3:.2f} us "
        f"({vb / (cold_v_ms / 1e3) / 1e9:.0f} GB/s)")

    # ---- CPU baseline: the oracle on the same input (FP64 upcast of X)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        O.build(force=False)
        m = O.Mesh.from_tissue(t)
        Xh = X.double().cpu().numpy()
        pin = g.uniform_params(t, P0=3.75)
        pin.lam = lam.double().cpu().numpy()
        n = 0
        c0 = time.perf_counter()
        while True:
            O.energy_forces(m, Xh, pin)
            n += 1
            if time.perf_counter() - c0 > args.cpu_seconds:
                break
        dt = time.perf_counter() - c0
        cpu = {"value": t.n_vert * n / dt, "unit": "vertex-force evals/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{n} full FP64 energy+force evaluations of the same 1e6-cell tissue "
                         f"({dt:.1f} s, one host thread)"}
        log(f"oracle: {n} evaluations in {dt:.1f}s")

    secondary = None
    if not args.no_secondary:
        from paper_2604_06896_amd import suite
        del F2, coeffs
        torch.cuda.empty_cache()
        secondary = {}
        w0 = time.perf_counter()
        secondary["batched_relax"] = suite.batched_relax(
            n_tissue=args.batch_tissues, max_iter=args.batch_max_iter,
            plain_sample=args.plain_sample, block_threads=1024, log=log)
        secondary["param_gradients"] = suite.param_gradients(
            n_tissue=args.grad_tissues, plain_sample=args.plain_sample, log=log)
        log(f"secondary measurements took {time.perf_counter() - w0:.1f}s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "vertex-force evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
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
        "roofline": {"bound": "hbm", "kernel": "k_vertex (vertex pass)",
                     "achieved": v_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": v_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": vb, "us_per_launch": v_ms * 1e3,
                     "cell_pass": {"achieved": c_gbs, "bytes_per_launch": cb,
                                   "us_per_launch": c_ms * 1e3},
                     "cold_caches": {"vertex_pass_us": cold_v_ms * 1e3,
                                     "vertex_pass_achieved": vb / (cold_v_ms / 1e3) / 1e9,
                                     "evaluation_us": cold_eval_ms * 1e3}},
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
