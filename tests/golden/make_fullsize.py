"""Write the full-length CPU-reference outputs that the full-size GPU parity
tests compare against (tests/golden/fullsize_<case>.npz).

Calls only the CPU reference (oracle/) on the seeded workload generators
(pd_inputs/).  For every case the reference runs the whole step count of
the workload and keeps, at n/4, n/2 and n steps:

  * the displacement and velocity of a fixed sample of nodes (caller order):
    8192 nodes drawn uniformly (numpy PCG64, seed 2309), the 2048 nodes with
    the largest damage (Eq. 1.31) at the end, and both ends of the bonds that
    came within 1e-5 of the critical stretch (up to 2048 nodes); the sample
    is the same at every snapshot (at most MAX_SAMPLE nodes, a seeded subset
    of that union if larger);
  * the norm of the full displacement vector;
  * every bond broken by the critical-stretch rule (Eq. 1.30) so far, as the
    sorted keys i * n + j of its caller nodes i < j (notch cuts excluded);
  * the bonds whose smallest breaking margin |s - s_c| / s_c so far is below
    1e-3, with that margin (the quantity the reading of several correct
    results compares a single-precision flip against).

and, at the end, the step at which each broken bond broke.  The meta record
holds the sizes, the time step, the critical stretch, the first break step,
the reference's own wall time and its thread count.

Stored form (compact): a broken set of at most KEEP_KEYS bonds is kept as
its sorted keys, delta-coded (brk_dkeys<k>, uint64), with the near-threshold
bonds and their margins (float32); every broken set is also kept as its size
(brk_count<k>) and the SHA-256 of its sorted keys as little-endian int64
(brk_sha<k>), which is what a comparison of sets too large to store uses.
The break steps are kept per bond for small final sets, else as a histogram
over 50-step bins (brk_hist).

usage: python -m tests.golden.make_fullsize [case ...] [--threads T]
       python -m tests.golden.make_fullsize --compact case ...   (re-encode a
           file written in the plain form)
       cases: impact3d cylinder3d cylinder3d_dx05 batch2d (default: all)
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import Oracle  # noqa: E402
from oracle import oracle as O  # noqa: E402
from pd_inputs import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = {
    # name: (generator, generator kwargs, steps)
    "impact3d": ("impact3d", {}, 2000),
    "cylinder3d": ("cylinder3d", {}, 5000),
    "cylinder3d_dx05": ("cylinder3d", {"dx": 0.5e-3}, 5000),
    "batch2d": ("batch2d", {}, 1000),
}

N_UNIFORM = 8192
N_DAMAGED = 2048
N_NEAR = 2048
MAX_SAMPLE = 12288
NEAR_SAMPLE = 1e-5
NEAR_KEEP = 1e-3


KEEP_KEYS = 250000


def keys_sha(keys: np.ndarray) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(np.sort(keys), dtype="<i8").tobytes()).hexdigest()


def compact(out: dict) -> dict:
    """The plain outputs of run_case in the stored form (see the module
    notes)."""
    meta = json.loads(str(out["meta"]))
    res = {k: v for k, v in out.items() if not k.startswith(("brk_keys", "near_keys", "near_margin", "brk_step"))}
    ns = res["sample"].size
    if ns > MAX_SAMPLE:
        keep = np.sort(np.random.Generator(np.random.PCG64(2309)).choice(ns, MAX_SAMPLE, replace=False))
        res["sample"] = res["sample"][keep]
        for k in range(len(meta["snapshots"])):
            res["u%d" % k] = res["u%d" % k][keep]
            res["v%d" % k] = res["v%d" % k][keep]
    for k in range(len(meta["snapshots"])):
        keys = np.asarray(out["brk_keys%d" % k], dtype=np.int64)
        res["brk_count%d" % k] = np.array(keys.size)
        res["brk_sha%d" % k] = np.array(keys_sha(keys))
        if keys.size <= KEEP_KEYS:
            res["brk_dkeys%d" % k] = np.diff(np.sort(keys), prepend=0).astype(np.uint64)
            nk = np.asarray(out["near_keys%d" % k], dtype=np.int64)
            o = np.argsort(nk)
            res["near_dkeys%d" % k] = np.diff(nk[o], prepend=0).astype(np.uint64)
            res["near_margin%d" % k] = np.asarray(out["near_margin%d" % k])[o].astype(np.float32)
    steps = np.asarray(out["brk_step"])
    if steps.size <= KEEP_KEYS:
        res["brk_step"] = steps.astype(np.int16)
    res["brk_hist"] = np.bincount(steps // 50, minlength=meta["steps"] // 50 + 1).astype(np.int64)
    return res


def load(case: str):
    """The stored outputs of a case: (arrays, meta), with brk_keys<k>,
    near_keys<k> decoded where stored."""
    g = dict(np.load(golden_path(case), allow_pickle=False))
    meta = json.loads(str(g["meta"]))
    for k in range(len(meta["snapshots"])):
        if "brk_dkeys%d" % k in g:
            g["brk_keys%d" % k] = np.cumsum(g["brk_dkeys%d" % k].astype(np.int64))
            g["near_keys%d" % k] = np.cumsum(g["near_dkeys%d" % k].astype(np.int64))
    return g, meta


def golden_path(case: str) -> str:
    return os.path.join(HERE, "fullsize_%s.npz" % case)


def workload(case: str):
    gen, kw, steps = CASES[case]
    return W.workload(gen, **kw), steps


def snapshots(steps: int):
    return [steps // 4, steps // 2, steps]


def run_case(case: str, log=print) -> dict:
    w, steps = workload(case)
    t0 = time.time()
    o = Oracle(w)
    t_setup = time.time() - t0
    bi, bj = o.bonds()
    keys_all = bi.astype(np.int64) * w.n + bj.astype(np.int64)
    o.track_bond_margins(True)
    u, v = o.initial_state()
    snaps = snapshots(steps)
    out = {}
    t_run = 0.0
    done = 0
    us, vs = [], []
    chunk = 50
    for k, target in enumerate(snaps):
        while done < target:
            n = min(chunk, target - done)
            t1 = time.time()
            o.run(n, u, v)
            t_run += time.time() - t1
            done += n
            brk = o.break_step()
            log("%s: step %d/%d, broken %d, %.1f s" % (case, done, steps, int((brk >= 0).sum()), t_run))
        brk = o.break_step()
        sel = brk >= 0
        out["brk_keys%d" % k] = np.sort(keys_all[sel])
        bm = o.bond_margins()
        near = bm < NEAR_KEEP
        out["near_keys%d" % k] = keys_all[near]
        out["near_margin%d" % k] = bm[near]
        out["unorm%d" % k] = np.array(np.linalg.norm(u))
        us.append(u.copy())
        vs.append(v.copy())
    brk = o.break_step()
    sel = brk >= 0
    order = np.argsort(keys_all[sel])
    out["brk_step"] = brk[sel][order].astype(np.int32)
    # the node sample
    rng = np.random.Generator(np.random.PCG64(2309))
    uni = rng.choice(w.n, size=min(N_UNIFORM, w.n), replace=False)
    phi = o.damage()
    dam = np.argsort(-phi, kind="stable")[:N_DAMAGED]
    dam = dam[phi[dam] > 0]
    bm = o.bond_margins()
    close = np.nonzero(bm < NEAR_SAMPLE)[0]
    close = close[np.argsort(bm[close], kind="stable")]
    ends = np.unique(np.concatenate([bi[close], bj[close]]))[:N_NEAR]
    sample = np.unique(np.concatenate([uni, dam, ends])).astype(np.int32)
    out["sample"] = sample
    for k in range(len(snaps)):
        out["u%d" % k] = us[k][sample]
        out["v%d" % k] = vs[k][sample]
    first = int(brk[sel].min()) if sel.any() else -1
    meta = dict(case=case, n=int(w.n), nb=int(o.nb), n_cut=int(o.n_cut), steps=steps, snapshots=snaps,
                dt=[float(x) for x in o.dt], s0=[float(x) for x in o.s0], first_break_step=first,
                broken=[int(out["brk_keys%d" % k].size) for k in range(len(snaps))],
                min_margin=float(o.min_margin()), n_close_1e6=int(o.n_close()),
                threads=int(O.num_threads()), setup_s=t_setup, run_s=t_run,
                bond_updates_per_s=float(o.nb) * steps / t_run if t_run > 0 else None)
    out["meta"] = np.array(json.dumps(meta))
    return out


def main(argv):
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=list(CASES))
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--compact", action="store_true")
    a = ap.parse_args(argv)
    if a.compact:
        for case in a.cases:
            out = dict(np.load(golden_path(case), allow_pickle=False))
            if "brk_count0" not in out:
                np.savez_compressed(golden_path(case), **compact(out))
            print("compact", golden_path(case), os.path.getsize(golden_path(case)), flush=True)
        return
    if a.threads > 0:
        O.set_num_threads(a.threads)
    for case in a.cases:
        out = compact(run_case(case, log=lambda s: print(s, flush=True)))
        np.savez_compressed(golden_path(case), **out)
        print("wrote", golden_path(case), json.loads(str(out["meta"])), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
