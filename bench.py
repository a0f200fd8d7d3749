#!/usr/bin/env python3
"""Throughput of the explicit linearized OSB-PD step on one MI355X.

A step is one pass of the whole hot path over the workload: breaking check
and dilatation (pass 1), pair force and explicit update (pass 2).  The value
is unique bonds x steps / wall time of K timed steps (inputs resident in
HBM, steps replayed from a captured hipGraph), in bond-updates/s.

Beside it the JSON line carries
  roofline     -- the dominant kernel's algorithmic bytes per launch divided
                  by its average duration (HIP events on the launch stream),
                  against the 8 TB/s HBM peak of MI355X;
  cpu_baseline -- the CPU reference timed on a bounded sample of the same
                  workload on this host's cores;
  fp64         -- the same workload with the double-precision force path.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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
# published MI355X vector peaks (TFLOP/s)
VALU_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}

WORKLOADS = {
    # name: (generator kwargs, description)
    "cylinder3d": (dict(), "3D notched cylinder under end twist, r=25 mm, L=100 mm, dx=0.6 mm, "
                           "delta=3.015 dx, helical notch, 911,319 nodes"),
    "cylinder3d_dx05": (dict(dx=0.5e-3), "3D notched cylinder, dx=0.5 mm, 1,572,000 nodes"),
    "impact3d": (dict(), "3D double-notched plate 200x200x9, 16.5 m/s edge impact, 360,000 nodes"),
    "plate2d": (dict(), "2D plane-stress edge-notched plate 200x80, 1 MPa, 16,000 nodes"),
    "batch2d": (dict(), "256 random 2D plane-stress notched plates (seed 2309), 5,800,669 nodes"),
    "cantilever3d": (dict(), "3D cantilever 20x4x4, 320 nodes"),
}


def make_workload(name):
    from pd_inputs import workloads as W
    kw, desc = WORKLOADS[name]
    gen = name.split("_")[0] if name.startswith("cylinder") else name
    return W.workload(gen, **kw), desc


def algorithmic_bytes(kernel: str, precision: str, nnz: int, n: int, n_loaded: int, tiled: bool,
                      dim: int = 3) -> int:
    """Bytes one launch must move between HBM and the chip (each array read
    or written once; neighbour data is served by the caches or LDS).

    Per directed bond: 1 bit of bond status (1/8 B), plus the 4 B bond word
    for the gather kernels; the LDS-staged tile kernels read no bond word
    (the stencil position of a bond gives its neighbour).  Per-row vectors
    (velocity v, the FP32 row constant D, the carried force parts) are stored
    with the dimension: w = 3 packed entries in 3D, 2 in 2D.
    Per node, gather kernels (pair force summed in pass 2):
      FP64 pass 1: u,V 32; aux 4; (theta/m, 1/m) 16 read + 8 write
      FP64 pass 2: u,V 32; (theta/m, 1/m) 16; aux 4; v 8w + 8w; u,V 32 write
      FP32 pass 1: shadow 16; aux 4; float (theta/m, 1/m) 8 + 4
      FP32 pass 2: shadow 16; float (theta/m, 1/m) 8; aux 4; D 8w; u,V 32;
                   v 8w + 8w; u,V 32 write; next shadow 16 write
    Per node, tile kernels (deviatoric part of the pair force in pass 1):
      FP64 pass 1: u,V 32; 1/m 8; aux 4; theta/m 8 write; force part 8w write
      FP64 pass 2: theta/m 8; u,V 32; aux 4; force part 8w; v 8w + 8w;
                   u,V 32 write
      FP32 pass 1: shadow 16; 1/m 4; aux 4; (theta/m, V) 8 write; force part
                   4w write
      FP32 pass 2: (theta/m, V) 8; aux 4; D 8w; force part 4w; u,V 32;
                   v 8w + 8w; u,V 32 write; next shadow 16 write
    Loaded nodes read their external force (32 B) in pass 2."""
    w = 3 if dim == 3 else 2
    bond = nnz * (0.125 if tiled else 4.125)
    if tiled:
        node = {("fp64", "pass1"): 52 + 8 * w, ("fp64", "pass2"): 76 + 24 * w,
                ("fp32", "pass1"): 32 + 4 * w, ("fp32", "pass2"): 92 + 28 * w}[(precision, kernel)]
    else:
        node = {("fp64", "pass1"): 60, ("fp64", "pass2"): 84 + 16 * w,
                ("fp32", "pass1"): 32, ("fp32", "pass2"): 108 + 24 * w}[(precision, kernel)]
    extra = 32 * n_loaded if kernel == "pass2" else 0
    return int(bond + node * n + extra)


def algorithmic_flops(kernel: str, nnz: int, tiled: bool) -> int:
    """Floating-point operations one launch must do, per directed bond (the
    per-node update is negligible beside them):
      extension M.(u_j - u_i): 3 sub + 3 mul + 2 add = 8; stretch test 1;
      dilatation term x e V_j: 2 mul + 1 add = 3;
      deviatoric force G e (1/m_i + 1/m_j) V_j M: 1 add + 2 mul + 3 mul + 3 add = 9;
      dilatational force (K - G/3) x (q_i + q_j) V_j M: 1 add + 2 mul + 6 = 9.
    Tile kernels: pass 1 = 8 + 1 + 3 + 9 = 21, pass 2 = 9.  Gather kernels:
    pass 1 = 8 + 1 + 3 = 12; pass 2 recomputes the extension and sums the
    whole bracket [(K - G/3) x (q_i + q_j) + G e (1/m_i + 1/m_j)] V_j M:
    8 + 3 + 3 + 1 (sum) + 1 (V_j) + 6 (M, accumulate) = 22."""
    per = {("pass1", True): 21, ("pass2", True): 9, ("pass1", False): 12, ("pass2", False): 22}[(kernel, tiled)]
    return per * nnz


def traffic_from_profiles(kernel_name: str, src_hash: str):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/
    traffic.json) as (FETCH_SIZE and WRITE_SIZE each scaled by a copy of
    known size, the same reads counted by request size), each None if absent
    or taken on a different kernel source.  The second is exact: FETCH_SIZE
    counts a 128-byte read request as 64 bytes on gfx950, so the copy's
    scale (2) overstates kernels that also issue 64-byte requests."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel_name)
    if not e or e.get("source_sha") != src_hash:
        return None, None
    return e.get("bytes_per_launch"), e.get("bytes_per_launch_exact")


def roofline_entry(s, args, dom, ms1, ms2, nnz, n, n_loaded):
    """Roofline of the dominant kernel: the ceiling that binds its algorithmic
    work (bytes at the HBM peak vs flops at the vector peak of its precision),
    the achieved fraction of it from the HIP-event duration, and the measured
    HBM traffic per launch when profiles/traffic.json holds it for this
    kernel source."""
    tiled = args.kernel != "gather" and s.tiled_supported(args.precision)
    kname = f"k_{'t' if tiled else ''}{dom}_{'f32' if args.precision == 'fp32' else 'f64'}"
    if tiled and args.kernel == "super" and args.precision == "fp32":
        kname += " (super-tiles)"
    if args.extension == "finite":
        kname = f"k_tpass{dom[-1]}_f64 (finite model)" if tiled else f"k_fin_{dom}"
    ms_dom = ms1 if dom == "pass1" else ms2
    sec = ms_dom * 1e-3
    byt = algorithmic_bytes(dom, args.precision, nnz, n, n_loaded, tiled, int(s.fam.sizes.dim))
    fl = algorithmic_flops(dom, nnz, tiled)
    if args.extension == "finite" and tiled:
        # per directed bond, tile kernels: deformed bond 6, |Y|^2 5, square
        # root 1, e 1, dilatation 3, reciprocal square root with its Newton
        # step 5, direction 3, deviatoric bracket 3 and accumulation 6 (pass
        # 1: 33); pass 2 rebuilds Y (6 + 5 + 5 + 3) and adds the dilatational
        # bracket 4 and accumulation 6 (29)
        fl = (33 if dom == "pass1" else 29) * nnz
    elif args.extension == "finite":
        # per directed bond, bond-list kernels: deformed bond 6, |Y| 5 +
        # sqrt, e 1, stretch 1, dilatation 3 (pass 1: 20 with eta 3); pass 2
        # adds Y/|Y| 3 and the bracket and accumulation 13 (31)
        fl = (20 if dom == "pass1" else 31) * nnz
    peak_fl = VALU_PEAK_TFLOPS[args.precision]
    gbs, tfs = byt / sec / 1e9, fl / sec / 1e12
    alu = fl / (peak_fl * 1e12) > byt / (HBM_PEAK_GBS * 1e9)
    from paper_2309_11273_amd.profsum import kernel_source_hash
    traffic, traffic_exact = (None, None) if args.extension == "finite" else \
        traffic_from_profiles(f"{kname}@{args.workload}", kernel_source_hash(kname.split(" ")[0]))
    return {"bound": "alu" if alu else "hbm",
            "achieved": round(tfs if alu else gbs, 2), "peak": peak_fl if alu else HBM_PEAK_GBS,
            "unit": "TFLOP/s" if alu else "GB/s",
            "frac": round(tfs / peak_fl if alu else gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic, "traffic_exact": traffic_exact, "kernel": kname, "kernel_ms": round(ms_dom, 5),
            "algorithmic_bytes": byt, "algorithmic_flops": fl,
            "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "valu_tflops": round(tfs, 2), "valu_frac": round(tfs / peak_fl, 4),
            "pass1_ms": round(ms1, 5), "pass2_ms": round(ms2, 5)}


def fac_bytes(kernel: str, dim: int, nnz: int, nb: int, n: int, n_loaded: int) -> int:
    """Algorithmic bytes of one launch of a factored-scheme kernel: every
    stored value and column index of the operator it applies read once
    (double values, int32 columns), the vectors it multiplies read once, its
    result written once.

      k_fac_extension  E = C_e U: per bond 2 dim values, 2 columns, x_b,
                       the owner position, 1 status bit, E_b written;
                       U (32 B per node) read
      k_fac_dilatation Theta = C_theta E: per directed bond 1 value, 1 column;
                       E read; Theta written
      k_fac_force      F = K_theta Theta + K_e E and the update: per directed
                       bond 2 dim values, 2 columns; K_theta diagonal (8 dim
                       per node), Theta and E read; per node u,V (32 B), v
                       (8 dim), aux (4 B) read, u,V and v written; F_ext rows
    """
    if kernel == "k_fac_extension":
        return nb * (16 * dim + 8 + 8 + 4 + 8) + nnz // 8 + 32 * n
    if kernel == "k_fac_dilatation":
        return nnz * 12 + 8 * nb + 8 * n
    return nnz * (16 * dim + 8) + n * (8 * dim + 8 + (36 + 8 * dim) + (32 + 8 * dim)) + 8 * nb + 32 * n_loaded


def fac_roofline(ms, dim, nnz, nb, n, n_loaded, workload):
    """Roofline of the factored scheme's dominant kernel (HBM-bound: about
    two flops per 12 bytes of value and column)."""
    kname = max(ms, key=ms.get)
    byt = fac_bytes(kname, dim, nnz, nb, n, n_loaded)
    gbs = byt / (ms[kname] * 1e-3) / 1e9
    from paper_2309_11273_amd.profsum import kernel_source_hash
    traffic, traffic_exact = traffic_from_profiles(f"{kname}@{workload}", kernel_source_hash(kname))
    return {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_exact": traffic_exact,
            "kernel": kname,
            "kernel_ms": round(ms[kname], 5), "algorithmic_bytes": byt,
            "kernels_ms": {k: round(v, 5) for k, v in ms.items()},
            "kernels_gbs": {k: round(fac_bytes(k, dim, nnz, nb, n, n_loaded) / (v * 1e-3) / 1e9, 1)
                            for k, v in ms.items()}}


def time_gpu(s, steps, warmup, precision, form, chunk, kernel="auto", extension="linear", block=0):
    import torch
    s.step(warmup, precision=precision, form=form, graph_chunk=chunk, report=False, kernel=kernel,
           extension=extension, block=block)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, precision=precision, form=form, graph_chunk=chunk, report=False, kernel=kernel,
           extension=extension, block=block)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def golden_compare(s, name, step):
    """Error against the CPU reference at 'step' of the full workload, from
    the reference's stored full-length outputs (tests/golden/, written by the
    reference alone): relative L2 of the displacement over the stored node
    sample and the bonds on whose status the two runs differ.  None if no
    stored output covers this workload and step."""
    import hashlib

    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{name}.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path, allow_pickle=False)
    meta = json.loads(str(g["meta"]))
    if step not in meta["snapshots"]:
        return None
    k = meta["snapshots"].index(step)
    u, _ = s.read()
    idx = g["sample"]
    ur = g[f"u{k}"]
    keys_g = s.broken_keys()
    n_ref = int(g[f"brk_count{k}"])
    sha = hashlib.sha256(np.ascontiguousarray(np.sort(keys_g), dtype="<i8").tobytes()).hexdigest()
    out = {"step": step, "rel_l2_u_sample": float(np.linalg.norm(u[idx] - ur) / np.linalg.norm(ur)),
           "sample_nodes": int(idx.size), "broken_oracle": n_ref, "broken_gpu": int(keys_g.size),
           "broken_sets_identical": bool(keys_g.size == n_ref and sha == str(g[f"brk_sha{k}"])),
           "first_break_step_oracle": meta.get("first_break_step")}
    if f"brk_dkeys{k}" in g.files:
        keys_o = np.cumsum(g[f"brk_dkeys{k}"].astype(np.int64))
        out["bonds_differ"] = int(np.setxor1d(keys_o, keys_g).size)
    return out


def run_window(s, w, args, precision, preroll, chunk, extension="linear", kernel="auto", block=0):
    """Untimed pre-roll, warm-up, then the timed steps; returns the wall time
    of the timed steps and the step counter at their end."""
    import torch
    if preroll > 0:
        s.step(preroll, precision=precision, form=args.form, graph_chunk=chunk, report=False, kernel=kernel,
               extension=extension, block=block)
    el = time_gpu(s, args.steps, args.warmup, precision, args.form, chunk, kernel, extension, block)
    torch.cuda.synchronize()
    return el, preroll + args.warmup + args.steps


def default_preroll(args, w):
    """Untimed steps before the warm-up so that the timed window ends where
    the workload's run ends (for the cylinder: inside its fracture phase)."""
    if args.preroll >= 0:
        return args.preroll
    return max(0, int(w.steps) - args.warmup - args.steps)


def batch_baseline(n_plates, steps, chunk):
    """Wall time of 'steps' FP64 steps of every plate of the batch, one plate
    after the other, each with its own solver, context and captured graph."""
    import torch
    from paper_2309_11273_amd.solver import Context, Solver
    from pd_inputs import workloads as W
    solvers = [Solver(W.batch2d(n_plates=1, first=k), ctx=Context(0), fp32_state=False) for k in range(n_plates)]
    for s in solvers:
        s.step(chunk, precision="fp64", graph_chunk=chunk, report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps, precision="fp64", graph_chunk=chunk, report=False)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def time_static(s, steps, warmup, mf=False, use_k=True):
    """Wall time of 'steps' conjugate-gradient iterations (HIP events on the
    library's stream), less that of a solve with none (the start phase)."""
    import torch
    s.static_solve(tol=1e-300, max_iter=max(1, warmup), check_every=max(1, warmup), matrix_free=mf, use_K=use_k)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    u0 = s.uv[s.S.cur].clone()
    ev[0].record()
    s.static_solve(tol=1e-300, max_iter=1, check_every=1, matrix_free=mf, use_K=use_k)
    ev[1].record()
    s.uv[s.S.cur].copy_(u0)
    ev[2].record()
    s.static_solve(tol=1e-300, max_iter=steps + 1, check_every=steps + 1, matrix_free=mf, use_K=use_k)
    ev[3].record()
    torch.cuda.synchronize()
    return (ev[2].elapsed_time(ev[3]) - ev[0].elapsed_time(ev[1])) * 1e-3


def time_adr(s, steps, warmup, chunk, kernel="auto", extension="linear"):
    import torch
    s.adr_step(warmup, graph_chunk=chunk, report=False, kernel=kernel, extension=extension)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.adr_step(steps, graph_chunk=chunk, report=False, kernel=kernel, extension=extension)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(w, budget_s: float, mode: str = "step"):
    """The CPU reference timed on a bounded sample of the same workload and
    the same operation: explicit steps (mode "step"; also the reference of
    the factored form, which applies the same operator), explicit steps of
    the finite model ("finite"), or relaxation iterations ("adr")."""
    from oracle import Oracle
    from oracle.oracle import num_threads
    o = Oracle(w)
    if mode == "finite":
        o.set_finite(True)
    if mode == "adr":
        st = o.adr_start()
        advance = lambda: o.adr_run(1, st)  # noqa: E731
    else:
        u, v = o.initial_state()
        advance = lambda: o.run(1, u, v)  # noqa: E731
    advance()  # first touch
    n, t0 = 0, time.perf_counter()
    while True:
        advance()
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 1000:
            break
    what = {"step": "explicit steps", "finite": "explicit steps of the finite model",
            "adr": "relaxation iterations"}[mode]
    return dict(value=o.nb * n / el, unit="bond-updates/s", cores=num_threads(), kind="oracle",
                sample=f"{w.name}: {n} {what} of the full workload ({o.nb} unique bonds) "
                       f"after one untimed one, FP64 loop reference with OpenMP over nodes")


def leg_roofline(s, args, nnz, n, n_loaded):
    """Kernel durations of the FP32 tile path (HIP events, eager steps) and
    the roofline of its dominant kernel."""
    s.profile_read(reset=True)
    s.step(args.profile_steps, precision="fp32", profile=True, report=False)
    prof = s.profile_read(reset=True)
    ps = max(1, prof["steps"])
    ms1, ms2 = prof["ms_pass1"] / ps, prof["ms_pass2"] / ps
    a = argparse.Namespace(kernel="auto", precision="fp32", extension="linear", workload=args.workload)
    return roofline_entry(s, a, "pass2" if ms2 >= ms1 else "pass1", ms1, ms2, nnz, n, n_loaded)


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def batched_leg(args):
    """The 256-plate batch: FP32 force path, all plates in one launch per
    pass (graph replay), against plain FP64 run one plate at a time (each
    plate its own solver and graph), both over the same timed steps at the
    end of the 1000-step run."""
    import numpy as np
    import torch
    from paper_2309_11273_amd.solver import Solver
    progress("batched leg: 256 plates")
    w, desc = make_workload("batch2d")
    t0 = time.perf_counter()
    s = Solver(w, device=0)
    setup = time.perf_counter() - t0
    sz = s.fam.sizes
    nb, nnz = int(sz.n_bonds), int(sz.nnz)
    n_loaded = int(np.count_nonzero(np.abs(w.fext).sum(1)))
    a = argparse.Namespace(**vars(args))
    a.workload, a.form, a.kernel = "batch2d", "mf", "auto"
    pre = default_preroll(a, w)
    el, end = run_window(s, w, a, "fp32", pre, args.graph_chunk)
    err = golden_compare(s, "batch2d", end)
    st = s.step(0, precision="fp32")
    roof = leg_roofline(s, a, nnz, int(sz.n), n_loaded)
    s.reset()
    el64, _ = run_window(s, w, a, "fp64", pre, args.graph_chunk)
    del s
    torch.cuda.empty_cache()
    progress("batched leg: FP64 one plate at a time")
    el_b = batch_baseline(w.n_specimens, args.steps, args.graph_chunk)
    v32 = nb * args.steps / el
    return {"workload": desc, "nodes": int(sz.n), "unique_bonds": nb, "setup_s": round(setup, 2),
            "timed_window": [pre + args.warmup, pre + args.warmup + args.steps],
            "fp32_batched": {"value": v32, "ms_per_step": 1e3 * el / args.steps,
                             "broken_bonds_after_run": int(st["broken_total"]) // 2,
                             "fp64_rechecks": int(st["rechecks"]), "roofline": roof, "error_vs_oracle": err},
            "fp64_batched": {"value": nb * args.steps / el64, "ms_per_step": 1e3 * el64 / args.steps},
            "fp64_one_plate_at_a_time": {"value": nb * args.steps / el_b, "ms_per_step": 1e3 * el_b / args.steps},
            "fp32_batched_speedup_vs_fp64_one_at_a_time": v32 / (nb * args.steps / el_b),
            "fp32_batched_speedup_vs_fp64_batched": el64 / el}


def cylinder_dx05_leg(args):
    """The cylinder at dx = 0.5 mm (1,572,000 nodes), FP32 force path, timed
    at the end of its 5000-step run, with its own roofline."""
    import numpy as np
    from paper_2309_11273_amd.solver import Solver
    progress("cylinder dx 0.5 mm leg")
    w, desc = make_workload("cylinder3d_dx05")
    t0 = time.perf_counter()
    s = Solver(w, device=0)
    setup = time.perf_counter() - t0
    sz = s.fam.sizes
    nb, nnz = int(sz.n_bonds), int(sz.nnz)
    a = argparse.Namespace(**vars(args))
    a.workload, a.form, a.kernel = "cylinder3d_dx05", "mf", "auto"
    pre = default_preroll(a, w)
    el, end = run_window(s, w, a, "fp32", pre, args.graph_chunk)
    err = golden_compare(s, "cylinder3d_dx05", end)
    st = s.step(0, precision="fp32")
    roof = leg_roofline(s, a, nnz, int(sz.n), 0)
    return {"workload": desc, "nodes": int(sz.n), "unique_bonds": nb, "setup_s": round(setup, 2),
            "timed_window": [pre + args.warmup, pre + args.warmup + args.steps],
            "value": nb * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
            "broken_bonds_after_run": int(st["broken_total"]) // 2, "fp64_rechecks": int(st["rechecks"]),
            "roofline": roof, "error_vs_oracle": err}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="cylinder3d", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--form", default="mf", choices=["mf", "bsr", "fac"],
                    help="mf: matrix-free tile kernels; bsr: block-sparse K; fac: the paper's four "
                         "factored matrices (double values, so --precision fp64)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "gather", "tiled", "super", "tiled1"],
                    help="matrix-free kernels: auto (the library's tuner), gather (bond list), tiled (one tile "
                         "per workgroup in 3D, per wave in 2D), super (FP32: four tiles per workgroup sharing "
                         "one halo box), tiled1 (one tile per workgroup in 2D too)")
    ap.add_argument("--extension", default="linear", choices=["linear", "finite"],
                    help="finite: e = |x M + u_j - u_i| - x with the force along the deformed bond "
                         "(FP64 gather kernels)")
    ap.add_argument("--batch-baseline", action="store_true",
                    help="batch2d only: also time the plain FP64 path run one plate at a time (each plate "
                         "its own solver and graph), the baseline the batched form is compared with")
    ap.add_argument("--static", action="store_true",
                    help="time conjugate-gradient iterations of the static solve with the assembled "
                         "double block-sparse K (one K product per iteration)")
    ap.add_argument("--implicit", action="store_true",
                    help="implicit average-acceleration Newmark steps (dt = 10x the explicit one) solved "
                         "by conjugate gradients with the double block-sparse K")
    ap.add_argument("--matrix-free", action="store_true",
                    help="with --static / --implicit: CG products K p = -f(p) by the double force kernels "
                         "instead of the stored K (K then only gives the preconditioner's diagonal)")
    ap.add_argument("--no-stored-k", action="store_true",
                    help="with --matrix-free: assemble no K at all (the preconditioner's diagonal summed "
                         "from the bonds)")
    ap.add_argument("--adr", action="store_true",
                    help="time iterations of the adaptive dynamic relaxation (FP64 matrix-free force, "
                         "fictitious time step 1) instead of explicit steps")
    ap.add_argument("--graph-chunk", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--preroll", type=int, default=-1,
                    help="untimed steps before the warm-up; -1 (default): the workload's step count minus "
                         "warm-up and timed steps, so the timed window ends where the run does (the "
                         "cylinder's fracture phase) and the state can be compared with the stored "
                         "full-length reference outputs")
    ap.add_argument("--no-legs", action="store_true",
                    help="default run only: skip the batched (256 plates) and dx = 0.5 mm cylinder legs")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="size in MiB of the plain read+write kernel timed after the run (the HBM ceiling "
                         "and the known-size reference for the byte counters); 0 = 1024")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: only a single GPU is supported (asked for {max(args.gpus, world)}); the "
              "solver runs one GPU's share of the workload per process and has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2309_11273_amd.solver import Solver

    w, desc = make_workload(args.workload)
    if args.adr:
        # quasi-static loading: each relaxation iteration (fictitious time
        # step 1) moves the prescribed components by what one explicit step
        # of the dynamic run moves them
        dts = np.asarray(w.dt, dtype=np.float64).reshape(-1)
        w.v0 = w.v0 * dts[np.asarray(w.specimen)][:, None] if dts.size > 1 else w.v0 * float(dts[0])
        desc += "; prescribed displacement increment per iteration = one explicit step's"
    t_setup = time.perf_counter()
    s = Solver(w, device=0)
    setup_s = time.perf_counter() - t_setup
    sz = s.fam.sizes
    n_bonds, nnz = int(sz.n_bonds), int(sz.nnz)
    n_loaded = int(np.count_nonzero(np.abs(w.fext).sum(1)))
    if args.form == "bsr":
        s.build_K(fp32=(args.precision == "fp32"))
        s.assemble_K()
    if args.form == "fac":
        args.precision = "fp64"
        s.build_factored()
        s.assemble_factored()
    if args.extension == "finite":
        if args.form != "mf":
            sys.exit("bench.py: --extension finite runs with the matrix-free force (--form mf)")
        args.precision = "fp64"
    if args.adr:
        if args.form != "mf":
            sys.exit("bench.py: --adr runs with the matrix-free force (--form mf)")
        args.precision = "fp64"
        s.adr_setup(1.0)

    if args.static:
        args.precision = "fp64"
        # the static problem: prescribed components displaced by what 100
        # explicit steps of their prescribed velocity move them, plus the
        # external load
        dts = np.asarray(w.dt, dtype=np.float64).reshape(-1)
        s.reset(u0=w.v0 * (100.0 * (dts[np.asarray(w.specimen)][:, None] if dts.size > 1 else float(dts[0]))))
        use_k = not (args.matrix_free and args.no_stored_k)
        if use_k:
            s.build_K(fp32=False)
            s.assemble_K()
        el = time_static(s, args.steps, args.warmup, args.matrix_free, use_k)
        ms_it = 1e3 * el / args.steps
        kb = int(s.K_sizes.nnzb) if use_k else 0
        dim = int(sz.dim)
        # per iteration: the stored K's blocks and column indices, or the two
        # double force passes (84 + 172 B/node, 1/8 B/bond each), plus the
        # vector kernels (about 520 B/node)
        byt = (int(sz.n_pad) * (84 + 172 + 520) + nnz // 4) if args.matrix_free else \
            kb * (8 * dim * dim + 4) + int(sz.n_pad) * (8 + 512)
        gbs = byt / (ms_it * 1e-3) / 1e9
        out = {"metric": "bond-updates/s per explicit step", "value": n_bonds * args.steps / el,
               "unit": "bond-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": ms_it, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic",
               "config": {"workload": desc + "; static solve (prescribed components displaced by 100 explicit "
                                      "steps of their velocity), conjugate-gradient iterations (one K product each)",
                          "nodes": int(sz.n), "unique_bonds": n_bonds, "K_blocks": kb,
                          "operator": ("matrix-free (double force kernels)" + ("" if use_k else ", no stored K"))
                          if args.matrix_free else "stored K"},
               "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                            "kernel": "one CG iteration (block product + vector kernels)",
                            "kernel_ms": round(ms_it, 5), "algorithmic_bytes": byt}}
        print(json.dumps(out), flush=True)
        return
    if args.implicit:
        import torch
        args.precision = "fp64"
        use_k = not (args.matrix_free and args.no_stored_k)
        if use_k:
            s.build_K(fp32=False)
            s.assemble_K()
        dts = np.asarray(w.dt, dtype=np.float64).reshape(-1)
        dt_imp = 10.0 * float(dts.min())
        s.newmark_step(args.warmup, dt_imp, tol=1e-10, check_every=10, matrix_free=args.matrix_free, use_K=use_k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = s.newmark_step(args.steps, dt_imp, tol=1e-10, check_every=10, matrix_free=args.matrix_free,
                             use_K=use_k)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ms_step = 1e3 * el / args.steps
        its = rep["iterations"] / max(1, args.steps)
        kb = int(s.K_sizes.nnzb) if use_k else 0
        dim = int(sz.dim)
        byt = (int(sz.n_pad) * (84 + 172 + 520) + nnz // 4) if args.matrix_free else \
            kb * (8 * dim * dim + 4) + int(sz.n_pad) * (8 + 512)
        gbs = byt * its / max(1e-12, ms_step * 1e-3) / 1e9
        out = {"metric": "bond-updates/s per explicit step", "value": n_bonds * args.steps / el,
               "unit": "bond-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic",
               "config": {"workload": desc + "; implicit Newmark steps (average acceleration, dt = 10x the "
                                      "explicit step), CG to 1e-10 per step", "nodes": int(sz.n),
                          "unique_bonds": n_bonds, "K_blocks": kb, "cg_iterations_per_step": round(its, 2),
                          "operator": ("matrix-free (double force kernels)" + ("" if use_k else ", no stored K"))
                          if args.matrix_free else "stored K",
                          "converged": rep["converged"]},
               "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                            "kernel": "CG iterations of one step (block product + vector kernels, host "
                                      "convergence checks included)",
                            "kernel_ms": round(ms_step, 5), "algorithmic_bytes": int(byt * its)}}
        print(json.dumps(out), flush=True)
        return
    preroll = 0
    err_vs_oracle = None
    tune = None
    block = 0
    if args.kernel == "auto" and args.form == "mf" and not args.adr and args.extension == "linear":
        # the library's tuner picks the kernel kind (tile, super-tile, gather
        # at 64/128/256 threads) on this workload; the timed run uses its pick
        tune = s.autotune(args.precision, trial_steps=10)
        args.kernel = tune["kernel"] if tune["kernel"] != "auto" else "tiled"
        block = int(tune["block"])
    if args.adr:
        el = time_adr(s, args.steps, args.warmup, args.graph_chunk, args.kernel, args.extension)
    else:
        preroll = default_preroll(args, w)
        el, end_step = run_window(s, w, args, args.precision, preroll, args.graph_chunk, args.extension,
                                  args.kernel, block)
        if args.extension == "linear":
            err_vs_oracle = golden_compare(s, args.workload, end_step)
    ms_per_step = 1e3 * el / args.steps
    value = n_bonds * args.steps / el
    st_end = s.step(0, precision=args.precision, form=args.form) if not args.adr else None

    # kernel durations with HIP events on the launch stream
    s.profile_read(reset=True)
    if args.adr:
        s.adr_step(args.profile_steps, profile=True, report=False, kernel=args.kernel, extension=args.extension)
    else:
        s.step(args.profile_steps, precision=args.precision, form=args.form, profile=True, report=False,
               kernel=args.kernel, extension=args.extension, block=block)
    prof = s.profile_read(reset=True)
    ps = max(1, prof["steps"])
    ms1, ms2 = prof["ms_pass1"] / ps, prof["ms_pass2"] / ps
    dom = "pass2" if ms2 >= ms1 else "pass1"
    ms_dom = max(ms1, ms2)
    if args.form == "mf":
        roofline = roofline_entry(s, args, dom, ms1, ms2, nnz, int(sz.n), n_loaded)
        if args.adr:
            # pass 2 runs without its update here; the relaxation's own kernels
            roofline["relaxation_kernels_ms"] = round(prof["ms_extra"] / ps, 5)
    elif args.form == "bsr":
        # the block product with the update dominates; per block the values
        # (9 or 4 entries) and a column index, per row u, v, aux and the update
        dim = int(sz.dim)
        vb = 4 if args.precision == "fp32" else 8
        kb = int(s.K_sizes.nnzb)
        byt = kb * (dim * dim * vb + 4) + int(sz.n) * (8 + 32 + 68 + 64) + 32 * n_loaded
        gbs = byt / (ms2 * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_bsr_spmv",
                    "kernel_ms": round(ms2, 5), "algorithmic_bytes": byt, "K_blocks": kb,
                    "break_mark_ms": round(ms1, 5), "reassembly_ms": round(prof["ms_extra"] / ps, 5)}
    elif args.form == "fac":
        # pass 1: E product + breaking; extra: K_theta re-assembly check + Theta
        # product; pass 2: F product + update
        ms_fac = {"k_fac_extension": ms1, "k_fac_dilatation": prof["ms_extra"] / ps, "k_fac_force": ms2}
        roofline = fac_roofline(ms_fac, int(sz.dim), nnz, int(s.F.nb), int(sz.n), n_loaded, args.workload)
    else:
        roofline = None

    st = s.adr_step(0) if args.adr else st_end
    if args.adr:
        st["rechecks"] = 0
    out = {
        "metric": "bond-updates/s per explicit step",
        "value": value,
        "unit": "bond-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "nodes": int(sz.n), "unique_bonds": n_bonds, "directed_bonds": nnz,
                   "form": {"mf": "matrix-free", "bsr": "block-sparse K",
                            "fac": "factored matrices C_e, C_theta, K_theta, K_e"}[args.form]
                           + (", finite extension (Eqs. 1.10, 1.13)" if args.extension == "finite" else "")
                           + (", adaptive dynamic relaxation iterations" if args.adr else ""),
                   "state_dtype": "f64", "graph_chunk": args.graph_chunk, "setup_s": round(setup_s, 2),
                   "untimed_steps_before_warmup": preroll,
                   "timed_window": [preroll + args.warmup, preroll + args.warmup + args.steps],
                   "broken_bonds_after_run": int(st["broken_total"]) // 2,
                   "fp64_rechecks": int(st["rechecks"]),
                   "min_recheck_margin": st.get("min_margin")},
        "roofline": roofline,
        "error_vs_oracle": err_vs_oracle,
    }
    if tune is not None:
        out["config"]["kernel"] = args.kernel + (f" ({block} threads per block)" if args.kernel == "gather" else "")
        names = {1: "gather", 2: "tiled", 3: "super", 4: "tiled1"}
        out["autotune"] = {"pick": tune["kernel"], "block": tune["block"],
                           "candidates_ms_per_step": {f"{names.get(c['kernel'], c['kernel'])}"
                                                      f"{'/' + str(c['block']) if c['kernel'] == 1 else ''}":
                                                      round(c["ms"], 5) for c in tune["candidates"]}}
    if not args.no_fp64 and args.precision == "fp32":
        s.reset()
        el64, end64 = run_window(s, w, args, "fp64", preroll, args.graph_chunk)
        err64 = golden_compare(s, args.workload, end64)
        st64 = s.step(0, precision="fp64")
        s.profile_read(reset=True)
        s.step(args.profile_steps, precision="fp64", profile=True, report=False)
        p64 = s.profile_read(reset=True)
        ps = max(1, p64["steps"])
        out["fp64"] = {"value": n_bonds * args.steps / el64, "ms_per_step": 1e3 * el64 / args.steps,
                       "pass1_ms": p64["ms_pass1"] / ps, "pass2_ms": p64["ms_pass2"] / ps,
                       "broken_bonds_after_run": int(st64["broken_total"]) // 2, "error_vs_oracle": err64}
        out["fp32_speedup_vs_fp64"] = value / out["fp64"]["value"]
    del s
    torch.cuda.empty_cache()
    legs = (args.workload == "cylinder3d" and args.form == "mf" and args.precision == "fp32" and not args.adr
            and args.extension == "linear" and not args.no_legs)
    if legs:
        out["batched"] = batched_leg(args)
        torch.cuda.empty_cache()
        out["cylinder3d_dx05"] = cylinder_dx05_leg(args)
        torch.cuda.empty_cache()
    if args.batch_baseline and args.workload == "batch2d":
        el_b = batch_baseline(w.n_specimens, args.steps, args.graph_chunk)
        out["batch_baseline"] = {"kind": "plain FP64, one plate at a time",
                                 "ms_per_step": 1e3 * el_b / args.steps, "value": n_bonds * args.steps / el_b,
                                 "batched_speedup": value / (n_bonds * args.steps / el_b)}
        torch.cuda.empty_cache()
    # the practical HBM ceiling: a plain read-and-write kernel of known size
    # (also the reference the byte counters are scaled by)
    mb = args.copy_mb if args.copy_mb > 0 else 1024
    src = torch.ones(mb << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 2.0, out=dst)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        torch.mul(src, 2.0, out=dst)
    ev1.record()
    torch.cuda.synchronize()
    moved = 10 * 2 * src.numel() * 4
    out["copy_reference"] = {"read_bytes": src.numel() * 4, "write_bytes": dst.numel() * 4,
                             "gbs": round(moved / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 1)}
    del src, dst
    torch.cuda.empty_cache()
    if not args.no_cpu:
        progress("CPU baseline")
        mode = "adr" if args.adr else ("finite" if args.extension == "finite" else "step")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, mode)
        # the same reference on one core (a shorter sample: the rate per core)
        from oracle.oracle import num_threads, set_num_threads
        nt = num_threads()
        set_num_threads(1)
        try:
            out["cpu_baseline_1core"] = cpu_baseline(w, max(5.0, args.cpu_seconds / 2), mode)
        finally:
            set_num_threads(nt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
