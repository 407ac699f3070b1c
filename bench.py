"""Throughput of the SI-MLSDC / DG-SEM hot path on one MI355X.

Default workload: two-level SI-MLSDC for the 3-D compressible Navier-Stokes
Taylor-Green vortex on [0, 2 pi]^3, 16^3 hexahedra, fine P = 7 / M = 4,
coarse P = 3 / M = 2 (2.1 M nodes x 5 conserved variables on the fine
level; see paper_2504_18526_amd/workloads.py).  One step = one time step of
the method: cascade start, 3 V-cycles, fine post-sweep, every implicit
system solved by PCG to a relative residual of 1e-10.  Metric: fine-level
DOF-updates/s = nodes_fine * n_var * M_fine * fine_sweeps_per_step / (s / step).
`--workload burgers|convdiff|euler|batch` selects the other workloads.

Prints one JSON line with the contract fields plus `roofline` and
`cpu_baseline` (the CPU oracle on a bounded sample, rank 0, N = 1).  The
roofline kernel is the dominant kernel of the fine level's implicit solves,
timed with HIP events on the solver's stream around each of its launches in
the timed steps: the persistent PCG (one launch per Helmholtz solve) where
the fine level uses it, else the multi-kernel PCG's vector update (its
full-work launches; the matvec is reported beside it).
"""
import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the roofline kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) of
#   bench.py --no-cpu-baseline --variant-steps 0
# averaged over that kernel's dispatches and scaled by what the same counters
# read for a 256 MiB device copy (FETCH_SIZE reads half of the bytes a copy
# moves, WRITE_SIZE all of them).  A figure holds only for the kernel sources
# it was taken on (SHA-256 prefix of the files that build the kernel).
COUNTER_SCALE = {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
MEASURED_TRAFFIC = {
    # profiles/hbm_traffic_cg_iter_iso_ns3d_taylor_green_16x16x16_P7-3.md (full-work dispatches)
    ("ns3d_taylor_green_mlsdc_16^3_P7-3_M4-2", "k_cg_iter_iso<512>"):
        {"fetch_kib": 176087.4, "write_kib": 284908.7, "src": "c38f10cbdb2c0e1c"},
    # profiles/hbm_traffic_pcg_persistent_burgers2d_32x32_P8-4.md (the first 52 steps)
    ("burgers2d_mlsdc_32x32_P8-4_M5-3", "k_pcg_persistent<2,8,1>"):
        {"fetch_kib": 13661.7, "write_kib": 42690.7, "src": "97801ce289ad5faa"},
}
TRAFFIC_SOURCES = {
    "k_pcg_persistent": ["pcg_persistent.hip", "common.hpp", "xcd.hpp"],
    "k_sipg_apply": ["kernels.hip", "common.hpp", "xcd.hpp", "gll_const.hpp"],
    "k_sipg_apply_iso3": ["kernels.hip", "common.hpp", "xcd.hpp", "gll_const.hpp"],
    "k_sipg_apply_iso2": ["kernels.hip", "common.hpp", "xcd.hpp", "gll_const.hpp"],
    "k_cg_iter": ["kernels.hip", "common.hpp", "xcd.hpp", "gll_const.hpp"],
    "k_cg_iter_iso": ["kernels.hip", "common.hpp", "xcd.hpp", "gll_const.hpp"],
}


def strip_comments(src):
    """C++ source without its comments and blank-line differences: the digest
    follows the code the counters measured, not its wording."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def kernel_source_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    base = kernel.split("<")[0]
    for f in TRAFFIC_SOURCES[base]:
        with open(os.path.join(ROOT, "paper_2504_18526_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """Counter-measured HBM bytes per launch, or None when there is no
    measurement for this kernel source."""
    rec = MEASURED_TRAFFIC.get((workload, kernel))
    if rec is None or rec["src"] != kernel_source_digest(kernel):
        return None
    return int(1024 * (rec["fetch_kib"] * COUNTER_SCALE["FETCH_SIZE"] + rec["write_kib"] * COUNTER_SCALE["WRITE_SIZE"]))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's own count; 20 for the default workload)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps timed for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--reps", type=int, default=400, help="launches timed for the roofline kernel")
    ap.add_argument("--variant-steps", type=int, default=50,
                    help="steps timed for each of the mixed / learned variants (0: skip them)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (calibrates HBM byte counters)")
    ap.add_argument("--kernels-only", type=int, default=0, metavar="REPS",
                    help="only launch the fine level's CG matvec and vector update REPS times each, back to back "
                         "(for profiler counter runs), print their average times and exit")
    ap.add_argument("--net-forward-only", type=int, default=0, metavar="REPS",
                    help="only run the fine level's element network forward (BF16, then FP32) REPS times each on "
                         "all of its rows, hidden width --net-hidden (for MFMA counter runs), print times and exit")
    ap.add_argument("--net-hidden", type=int, default=256)
    ap.add_argument("--workload", default="ns",
                    help="ns (default: the two-level 3-D Navier-Stokes workload), burgers, convdiff, euler, "
                         "batch (64 independent instances)")
    return ap.parse_args()


def cpu_baseline(w, u0_path, gpu_step1_path, nsteps):
    """Time the CPU oracle on `nsteps` steps of workload `w` from the state in
    `u0_path`, in a child process with one BLAS/OpenMP thread (the paper's
    runs were single-threaded); the oracle's first step is compared with the
    GPU's in `gpu_step1_path`."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    code = f"""
import sys, time, json, numpy as np
sys.path.insert(0, {ROOT!r})
from oracle.sdc import DGLevel, MLSDC
from oracle.physics import Burgers, ConvDiff, Euler, NavierStokes
w = {json.dumps({k: v for k, v in w.items()})}
if w['eq'] == 'burgers':
    ph = Burgers(w['dim'], w['nu'])
elif w['eq'] == 'convdiff':
    ph = ConvDiff(list(w['a'][:w['dim']]), w['nu'])
elif w['eq'] == 'euler':
    ph = Euler(w['dim'], w['gamma'])
else:
    ph = NavierStokes(w['dim'], w['gamma'], w['mu'], w['Pr'])
lv = [DGLevel(ph, w['n_elem'], w['lo'], w['hi'], P, M, rtol=w['cg_rtol']) for P, M in zip(w['P'], w['M'])]
ml = MLSDC(list(reversed(lv)), n_coarse=w['n_coarse'], start=w['start'], cycles=w['cycles'],
           post_sweep=bool(w['post_sweep']), av=tuple(w['av']) if w.get('av') else None)
u = np.load({u0_path!r}).reshape(lv[0].mesh.shape(ph.nv))
g1 = np.load({gpu_step1_path!r}).reshape(u.shape)
t = time.perf_counter()
for k in range({nsteps}):
    u = ml.step(u, w['dt'])
    if k == 0:
        u1 = u.copy()
el = time.perf_counter() - t
err = float(np.linalg.norm(g1 - u1) / np.linalg.norm(u1))
print(json.dumps({{"seconds": el, "steps": {nsteps}, "rel_l2_step1": err}}))
"""
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        raise RuntimeError("cpu baseline failed: " + out.stderr[-2000:])
    return json.loads(out.stdout.strip().splitlines()[-1])


def ns_cpu_baseline(S, w, prob, meth, stream, dev, ne=4, nsteps=2):
    """The oracle on a bounded sample of the Navier-Stokes workload: `nsteps`
    time steps of the same two-level method (same degrees, nodes, start,
    cycles, CFL rule, initial data) on an ne^3-element mesh of the same
    domain, timed in a child process with one thread; the GPU steps the same
    sample from the same u0 and the first steps of both are compared."""
    import ctypes
    import numpy as np
    import torch
    from paper_2504_18526_amd.inputs import taylor_green
    from paper_2504_18526_amd.workloads import fine_sweeps_per_step, systems_dt
    ws = dict(w)
    ws["n_elem"] = (ne,) * w["dim"]
    ps = S.Problem()
    ctypes.memmove(ctypes.addressof(ps), ctypes.addressof(prob), ctypes.sizeof(S.Problem))
    for d in range(w["dim"]):
        ps.n_elem[d] = ne
    sv = S.Solver(ps, meth, stream=stream.cuda_stream)
    E, Np, nv, M = sv.level_info(0)
    x = sv.coords(0)
    u0 = np.ascontiguousarray(taylor_green([x[d] for d in range(w["dim"])], mach=w["mach"]).reshape(nv, E, Np))
    ws["dt"] = systems_dt(ws, u0)
    ud = torch.from_numpy(u0).to(dev)
    sv.set_state(ud)
    sv.step(ws["dt"])
    out = torch.empty_like(ud)
    sv.get_state(out)
    torch.cuda.synchronize()
    sv.close()
    with tempfile.TemporaryDirectory() as td:
        p0 = os.path.join(td, "u0.npy")
        p1 = os.path.join(td, "g1.npy")
        np.save(p0, u0)
        np.save(p1, out.cpu().numpy())
        r = cpu_baseline(ws, p0, p1, nsteps)
    dofu = E * Np * nv * M * fine_sweeps_per_step(ws) * r["steps"]
    return {"value": dofu / r["seconds"], "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{r['steps']} time steps of the same two-level method (P {w['P']}, M {w['M']}, cascade, "
                      f"{w['cycles']} V-cycles + post-sweep, CFL {w['cfl']}, Taylor-Green data, oracle CG to the same "
                      f"1e-10 tolerance) on a {ne}^3-element mesh of the same domain ({E * Np * nv} DOF, 1/"
                      f"{(w['n_elem'][0] // ne) ** w['dim']} of the workload), {r['seconds']:.1f} s",
            "gpu_vs_oracle_rel_l2_step1": r["rel_l2_step1"]}


def cpu_baseline_batch(inst, budget_s=15.0):
    """The CPU oracle (one thread) on a bounded sample of the batch: one step
    of each instance, smallest first, until the budget is spent."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    order = sorted(range(len(inst)), key=lambda i: inst[i]["n_elem"][0] ** 2 * (inst[i]["P"][0] + 1) ** 2)
    code = f"""
import sys, time, json, numpy as np
sys.path.insert(0, {ROOT!r})
from oracle.sdc import DGLevel, MLSDC
from oracle.physics import Burgers, ConvDiff
from paper_2504_18526_amd.inputs import burgers_field, convdiff_field
inst = {json.dumps([inst[i] for i in order])}
done, tot, dofu = [], 0.0, 0.0
for w in inst:
    ph = Burgers(2, w['nu']) if w['eq'] == 'burgers' else ConvDiff(list(w['a'][:2]), w['nu'])
    lv = [DGLevel(ph, w['n_elem'], w['lo'], w['hi'], P, M, rtol=w['cg_rtol']) for P, M in zip(w['P'], w['M'])]
    ml = MLSDC(list(reversed(lv)), n_coarse=w['n_coarse'], start=w['start'], cycles=w['cycles'],
               post_sweep=bool(w['post_sweep']))
    xs = lv[0].coords()
    f = convdiff_field if w['eq'] == 'convdiff' else burgers_field
    u = f([xs[0], xs[1]], seed=w['seed'], kmax=w['kmax'])[None]
    t = time.perf_counter()
    ml.step(u, w['dt'])
    tot += time.perf_counter() - t
    n1 = w['P'][0] + 1
    dofu += w['n_elem'][0] * w['n_elem'][1] * n1 * n1 * w['M'][0] * (w['cycles'] + w['post_sweep'])
    done.append(w['name'])
    if tot > {budget_s}:
        break
print(json.dumps({{"seconds": tot, "dof_updates": dofu, "instances": done}}))
"""
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    if out.returncode != 0:
        raise RuntimeError("cpu baseline failed: " + out.stderr[-2000:])
    return json.loads(out.stdout.strip().splitlines()[-1])


def main_batch(a, w):
    """The batched serving-shape workload: every instance stepped by the
    batch API (one handle and stream per instance), tuned by the library's
    autotuner first; whole-batch steps timed by the host clock between
    device synchronisations (the instances run on many streams)."""
    import numpy as np
    import torch
    from paper_2504_18526_amd import sisdc as S
    from paper_2504_18526_amd.inputs import burgers_field, convdiff_field
    from paper_2504_18526_amd.workloads import fine_sweeps_per_step
    inst = w["instances"]
    steps = a.steps if a.steps is not None else w["steps"]
    dev = torch.device("cuda:0")
    probs, meths = [], []
    for wi in inst:
        eqc = S.EQ_CONVDIFF if wi["eq"] == "convdiff" else S.EQ_BURGERS
        probs.append(S.make_problem(2, wi["n_elem"], wi["lo"], wi["hi"], eqc, a=wi["a"][:2], nu=wi["nu"]))
        meths.append(S.make_method(wi["P"], wi["M"], start=S.START_CASCADE, n_coarse_sweeps=wi["n_coarse"],
                                   post_sweep=wi["post_sweep"], n_iter=wi["cycles"], cg_rtol=wi["cg_rtol"],
                                   cg_maxit=2000, precision=S.MIXED if wi["precision"] == "mixed" else S.FP64))
    batch = S.Batch(probs, meths)
    dof_updates, fine_dof = 0.0, 0
    for i, wi in enumerate(inst):
        m = batch[i]
        E, Np, nv, M = m.level_info(0)
        x = m.coords(0)
        f = convdiff_field if wi["eq"] == "convdiff" else burgers_field
        u0 = np.ascontiguousarray(f([x[0], x[1]], seed=wi["seed"], kmax=wi["kmax"])[None].reshape(nv, E, Np))
        m.set_state(torch.from_numpy(u0).to(dev))
        dof_updates += E * Np * nv * M * fine_sweeps_per_step(wi)
        fine_dof += E * Np * nv
    dts = [wi["dt"] for wi in inst]
    t0 = time.perf_counter()
    threads, variants, precs, graph = batch.tune(dts, full=True)
    tune_s = time.perf_counter() - t0
    step1 = None
    for k in range(max(1, a.warmup)):
        batch.step(dts)
        if k == 0:
            step1 = []
            for i in range(len(inst)):
                E, Np, nv, M = batch[i].level_info(0)
                out = torch.empty(nv * E * Np, dtype=torch.float64, device=dev)
                batch[i].get_state(out)
                step1.append(out.cpu().numpy())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = {"cg_iters": 0, "solves": 0, "not_converged": 0, "ir_rounds": 0}
    for _ in range(steps):
        for st in batch.step(dts):
            for k in tot:
                tot[k] += st[k]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1000.0 * wall / steps
    value = dof_updates / (ms_step / 1000.0)

    # roofline: the multi-kernel PCG kernels of the largest instance
    big = max(range(len(inst)), key=lambda i: inst[i]["n_elem"][0] ** 2 * (inst[i]["P"][0] + 1) ** 2)
    wb = inst[big]
    Eb, Npb, nvb, Mb = batch[big].level_info(0)
    nf = wb["P"][0] + 1
    traces = 4 * nf / Npb
    reads_ub = 1.0 if wb["eq"] == "burgers" else 0.0
    kern = {}
    for key, kid, name, words in (
            ("matvec", S.K_SIPG_APPLY, f"k_sipg_apply<2,{wb['P'][0]}>", 2.0 + reads_ub + traces),
            ("update", S.K_CG_UPDATE, f"k_cg_iter<2,{wb['P'][0]}>", 12.0 + reads_ub + traces)):
        us = batch[big].profile_kernel(kid, 0, wb["dt"] / Mb, reps=a.reps)
        nbytes = 8.0 * words * Eb * Npb * nvb
        kern[key] = {"kernel": name, "avg_launch_us": round(us, 3), "algo_bytes_per_launch": int(nbytes),
                     "achieved_GBs": round(nbytes / (us * 1e-6) / 1e9, 1)}
    dom = max(kern.values(), key=lambda k: k["avg_launch_us"])
    other = kern["update"] if dom is kern["matvec"] else kern["matvec"]
    roofline = {"bound": "hbm", "achieved": dom["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom["achieved_GBs"] / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": dom["kernel"] + f" (largest instance, {wb['n_elem'][0]}^2 elements)",
                "avg_launch_us": dom["avg_launch_us"], "algo_bytes_per_launch": dom["algo_bytes_per_launch"],
                "other": other}

    cpu = None
    if not a.no_cpu_baseline:
        r = cpu_baseline_batch(inst)
        cpu = {"value": r["dof_updates"] / r["seconds"], "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"one step of each of the {len(r['instances'])} smallest instances, {r['seconds']:.1f} s"}
    rec = {
        "metric": "fine-level DOF-updates/s (s/step at fixed PCG tolerance 1e-10)",
        "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": steps, "warmup": a.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if all(p == S.FP64 for p in precs) else "f64 (FP32 inner PCG where tuned)",
        "data": "synthetic (seeded Fourier initial data)",
        "config": {"workload": w["name"], "instances": len(inst), "fine_dof": fine_dof, "global_batch": len(inst),
                   "seq_len": None, "parallelism": "none", "host_threads": threads,
                   "persistent_pcg_instances": int(sum(1 for v in variants if v == S.CG_AUTO)),
                   "fp64_instances": int(sum(1 for p in precs if p == S.FP64)), "step_graphs": bool(graph),
                   "tune_s": round(tune_s, 2), "cg_iters_per_step": tot["cg_iters"] / steps,
                   "ir_rounds_per_step": tot["ir_rounds"] / steps, "not_converged": tot["not_converged"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    batch.close()


def single_instance_rate(S, w, prob, meth, u0, dt, steps, warmup, dof_updates, stream):
    """One instance of a stacked ensemble stepped through its own handle:
    ms per step and fine-level DOF-updates/s, timed as the ensemble is."""
    import ctypes
    import torch
    p1 = S.Problem()
    ctypes.memmove(ctypes.byref(p1), ctypes.byref(prob), ctypes.sizeof(prob))
    p1.stack = 1
    sv = S.Solver(p1, meth, stream=stream.cuda_stream)
    ud = torch.from_numpy(u0.copy()).cuda()
    sv.set_state(ud)
    for _ in range(max(1, warmup)):
        sv.step(dt)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
    for _ in range(steps):
        sv.step(dt)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    sv.close()
    return {"ms_per_step": ms, "value": dof_updates / (ms / 1000.0), "unit": "DOF-updates/s"}


def run_variants(S, w, prob, stream, u0, dt, nsteps, dof_updates, start):
    """Plain FP64 vs mixed precision vs the learned initial guess (and both),
    and, on the systems' isotropic levels, vs the element-block Jacobi
    preconditioner by fast diagonalisation, each from the same state after
    the same warm-up, same PCG tolerance.
    The network of each level is trained on rows harvested from the plain
    solves of the warm-up steps (its training time is reported, not timed)."""
    import time
    import torch
    out = {}
    ref = None
    iso = w["eq"] in ("euler", "ns")  # the block-Jacobi (fast-diagonalisation) preconditioner applies there
    cases = [("plain_fp64", S.FP64, False, S.PRECOND_JACOBI), ("mixed", S.MIXED, False, S.PRECOND_JACOBI),
             ("learned_fp64", S.FP64, True, S.PRECOND_JACOBI), ("learned_mixed", S.MIXED, True, S.PRECOND_JACOBI)]
    if iso:
        cases.append(("fds_fp64", S.FP64, False, S.PRECOND_FDS))
    for name, prec, learned, pc in cases:
        meth = S.make_method(w["P"], w["M"], start=start, n_coarse_sweeps=w["n_coarse"],
                             post_sweep=w["post_sweep"], n_iter=w["cycles"], cg_rtol=w["cg_rtol"],
                             cg_maxit=1000, precision=prec, precond=pc)
        sv = S.Solver(prob, meth, stream=stream.cuda_stream)
        sv.set_state(u0)
        train_s = 0.0
        if learned:
            for lvl in range(len(w["P"])):
                sv.net_init(lvl, 64, seed=1 + lvl, max_batch=2048, max_rows=65536)
                sv.net_harvest(lvl, 1)
        for _ in range(2):
            sv.step(dt)
        if learned:
            t0 = time.perf_counter()
            for lvl in range(len(w["P"])):
                sv.net_harvest(lvl, 0)
                sv.net_train(lvl, 20, 512, 1e-3)
                sv.net_use(lvl, 1)
            torch.cuda.synchronize()
            train_s = time.perf_counter() - t0
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        its, rej, rounds = 0, 0, 0
        for _ in range(nsteps):
            st = sv.step(dt)
            its += st["cg_iters"]
            rej += st["net_rejected"]
            rounds += st["ir_rounds"]
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / nsteps
        fin = torch.empty_like(u0)
        sv.get_state(fin)
        if ref is None:
            ref = fin.clone()
        diff = float(torch.linalg.norm(fin - ref) / torch.linalg.norm(ref))
        out[name] = {"ms_per_step": ms, "dof_updates_per_s": dof_updates / (ms / 1000.0),
                     "cg_iters_per_step": its / nsteps, "rel_l2_vs_plain": diff,
                     "rejected_guesses": rej, "ir_rounds_per_step": rounds / nsteps, "train_s": train_s}
        sv.close()
    base = out["plain_fp64"]["ms_per_step"]
    for k in out:
        out[k]["speedup_vs_plain"] = base / out[k]["ms_per_step"]
    out["steps"] = nsteps
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus must be 1 (the sharded design is described, not run)"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2504_18526_amd import sisdc as S
    from paper_2504_18526_amd.inputs import burgers_field
    from paper_2504_18526_amd.workloads import fine_sweeps_per_step

    from paper_2504_18526_amd.inputs import convdiff_field, convdiff_exact, isentropic_vortex, taylor_green, sod_pair
    from paper_2504_18526_amd.workloads import WORKLOADS, systems_dt
    w = WORKLOADS[a.workload]()
    if w["eq"] == "batch":
        return main_batch(a, w)
    if a.steps is None:
        a.steps = w.get("steps", 200)
    dev = torch.device("cuda:0")
    if a.copy_probe_mb > 0:
        src = torch.empty(a.copy_probe_mb * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.Stream(device=dev)
    eqc = {"convdiff": S.EQ_CONVDIFF, "burgers": S.EQ_BURGERS, "euler": S.EQ_EULER, "ns": S.EQ_NS}[w["eq"]]
    B = w.get("stack", 1)
    prob = S.make_problem(w["dim"], w["n_elem"], w["lo"], w["hi"], eqc, a=w.get("a", (0.0, 0.0, 0.0)),
                          nu=w.get("nu", 0.0), gamma=w.get("gamma", 1.4), mu=w.get("mu", 0.0),
                          Pr=w.get("Pr", 0.71), stack=B)
    start = {"cascade": S.START_CASCADE, "fmg": S.START_FMG}[w["start"]]
    meth = S.make_method(w["P"], w["M"], start=start, n_coarse_sweeps=w["n_coarse"],
                         post_sweep=w["post_sweep"], n_iter=w["cycles"], cg_rtol=w["cg_rtol"],
                         cg_maxit=w.get("cg_maxit", 1000), av=w.get("av"), conserve=w.get("conserve", 1))
    sv = S.Solver(prob, meth, stream=stream.cuda_stream)
    E, Np, nv, M = sv.level_info(0)
    x = sv.coords(0)
    xs = [x[d] for d in range(w["dim"])]
    if w["eq"] == "burgers" and B > 1:  # instance k: seed + k, on its own box
        Ei = E // B
        xi = [c.reshape(B, Ei * Np) for c in xs]
        u0 = np.concatenate([burgers_field([c[k] for c in xi], seed=w["seed"] + k, kmax=w["kmax"])
                             for k in range(B)])[None]
    elif w["eq"] == "burgers":
        u0 = burgers_field(xs, seed=w["seed"], kmax=w["kmax"])[None]
    elif w["eq"] == "convdiff":
        u0 = convdiff_field(xs, seed=w["seed"], kmax=w["kmax"])[None]
    elif w.get("init") == "sod":
        u0 = sod_pair(xs, (w["hi"][0] - w["lo"][0]) / w["n_elem"][0], gamma=w["gamma"])
    elif w["eq"] == "euler":
        u0 = isentropic_vortex(xs)
    else:
        u0 = taylor_green(xs, mach=w["mach"])
    u0 = np.ascontiguousarray(u0.reshape(nv, E, Np))
    if "dt" not in w:
        w["dt"] = systems_dt(w, u0)
    ud = torch.from_numpy(u0).to(dev)
    sv.set_state(ud)
    dt = w["dt"]
    if a.net_forward_only > 0:
        rows = nv * E
        sv.net_init(0, a.net_hidden, seed=1, max_batch=rows, max_rows=rows)
        gen = torch.Generator(device=dev).manual_seed(5)
        X = torch.randn(rows, Np, dtype=torch.float32, device=dev, generator=gen)
        Y = torch.empty_like(X)
        rec = {"workload": w["name"], "rows": rows, "inputs": Np, "hidden": a.net_hidden}
        for name, bf16 in (("bf16_ms", True), ("fp32_ms", False)):
            sv.net_forward(0, X, Y, bf16=bf16)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.net_forward_only):
                sv.net_forward(0, X, Y, bf16=bf16)
            torch.cuda.synchronize()
            rec[name] = 1000.0 * (time.perf_counter() - t0) / a.net_forward_only
        print(json.dumps(rec), flush=True)
        sv.close()
        return
    if a.kernels_only > 0:
        sv.update_step_params()
        rec = {"workload": w["name"], "dt_m": dt / M}
        for key, kid in (("matvec_us", S.K_SIPG_APPLY), ("update_us", S.K_CG_UPDATE)):
            rec[key] = sv.profile_kernel(kid, 0, dt / M, reps=a.kernels_only)
        print(json.dumps(rec), flush=True)
        sv.close()
        return

    # warm-up (the first warm-up step is kept for the parity check against the oracle)
    step1 = None
    for k in range(max(1, a.warmup)):
        sv.step(dt)
        if k == 0:
            out = torch.empty_like(ud)
            sv.get_state(out)
            step1 = out.cpu().numpy()

    # events around every persistent PCG launch of the timed steps, and
    # around the launches of every 8th multi-kernel solve (an event costs
    # several microseconds of queue work; timing every solve would slow the
    # timed steps by several per cent)
    sv.pcg_timing(True, stride=8)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
    t0 = time.perf_counter()
    tot = {"cg_iters": 0, "solves": 0, "fine_sweeps": 0, "not_converged": 0, "max_rel_residual": 0.0}
    step_ev = []  # an event after every step, for the median step time
    for _ in range(a.steps):
        st = sv.step(dt)
        for k in ("cg_iters", "solves", "fine_sweeps", "not_converged"):
            tot[k] += st[k]
        tot["max_rel_residual"] = max(tot["max_rel_residual"], st["max_rel_residual"])
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        step_ev.append(e)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / a.steps
    per_step = [ev0.elapsed_time(step_ev[0])] + [step_ev[k - 1].elapsed_time(step_ev[k]) for k in range(1, a.steps)]
    ms_median = float(np.median(per_step))
    # error against the exact solution where the problem has one
    err_exact = None
    if w["eq"] in ("euler", "convdiff") and w.get("init") != "sod" and B == 1:
        t_end = (max(1, a.warmup) + a.steps) * dt
        fin = torch.empty_like(ud)
        sv.get_state(fin)
        if w["eq"] == "euler":
            ex = isentropic_vortex(xs, t=t_end)
        else:
            ex = convdiff_exact(xs, t_end, w["a"], w["nu"], seed=w["seed"], kmax=w["kmax"])
        ex = np.ascontiguousarray(np.asarray(ex).reshape(nv, E, Np))
        fv = fin.cpu().numpy()
        err_exact = float(np.linalg.norm(fv - ex) / np.linalg.norm(ex))

    sweeps = fine_sweeps_per_step(w)
    dof_updates = E * Np * nv * M * sweeps
    value = dof_updates / (ms_step / 1000.0)

    # roofline of the dominant kernel, from the events recorded around its
    # launches in the timed steps
    pcg_n, pcg_it, pcg_us = sv.pcg_timing_get(0)
    up_n, up_us = sv.cg_kernel_timing_get(0, S.K_CG_UPDATE)
    mv_n, mv_us = sv.cg_kernel_timing_get(0, S.K_SIPG_APPLY)
    sv.pcg_timing(False)
    fine_dof = E * Np * nv
    nf = (w["P"][0] + 1) ** (w["dim"] - 1)  # face nodes per element face
    traces = 2 * w["dim"] * nf / Np         # face-trace words per DOF
    iso = w["eq"] in ("euler", "ns") and (w["dim"] == 2 or w["P"][0] in (1, 3, 7)) and not w.get("av")
    if iso:
        # isotropic kernels: the matvec reads r (scaled in-kernel to z) and
        # writes w; the update reads r, w, p, s and writes r, p, s, and on odd
        # iterations also x (read + write): 8 words per DOF on average over
        # the launches of a solve.
        mv_words, up_words = 2.0, 8.0
        mv_name = f"k_sipg_apply_iso{w['dim']}<{w['P'][0]}>"
        up_name = f"k_cg_iter_iso<{Np}>"
    else:
        reads_ub = 1.0 if w["eq"] == "burgers" else 0.0  # the coefficient state (Burgers only)
        mv_words = 2.0 + reads_ub + traces                 # read z (+ u_b), traces; write w
        up_words = 12.0 + reads_ub + traces                # z, w, p, s, x, r, diag in; p, s, x, r, z, traces out
        mv_name = f"k_sipg_apply<{w['dim']},{w['P'][0]}>"
        up_name = f"k_cg_iter<{w['dim']},{w['P'][0]}>"

    def kern_rec(name, words, n, us):
        nbytes = 8.0 * words * fine_dof
        avg = us / n if n > 0 else float("nan")
        return {"kernel": name, "launches": n, "avg_launch_us": round(avg, 3), "algo_bytes_per_launch": int(nbytes),
                "achieved_GBs": round(nbytes / (avg * 1e-6) / 1e9, 1) if n > 0 else None}

    matvec = kern_rec(mv_name, mv_words, mv_n, mv_us)
    update = kern_rec(up_name, up_words, up_n, up_us)
    if pcg_n > 0:
        # the persistent PCG: one launch = one whole fine-level Helmholtz solve.
        # Algorithmic bytes of a streaming PCG: 5 FP64 words per DOF to set up
        # a solve and 11 per iteration (fused matvec / dot / update).
        name = f"k_pcg_persistent<{w['dim']},{w['P'][0]},{nv}>"
        algo = 8.0 * fine_dof * (5.0 * pcg_n + 11.0 * pcg_it)
        achieved = algo / (pcg_us * 1e-6) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(w["name"], name),
                    "kernel": name + " (whole fine-level PCG solve)",
                    "avg_launch_us": round(pcg_us / pcg_n, 3), "launches": pcg_n,
                    "iters_per_launch": round(pcg_it / pcg_n, 3),
                    "algo_bytes_per_launch": int(algo / pcg_n), "timing": "HIP events around every launch of the timed steps"}
    else:
        # multi-kernel PCG: the kernel with the larger summed time dominates
        # (both run once per iteration)
        dom, other = (update, matvec) if up_us >= mv_us else (matvec, update)
        roofline = {"bound": "hbm", "achieved": dom["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(dom["achieved_GBs"] / HBM_PEAK_GBS, 4) if dom["achieved_GBs"] else None,
                    "traffic": measured_traffic(w["name"], dom["kernel"]),
                    "kernel": dom["kernel"], "avg_launch_us": dom["avg_launch_us"], "launches": dom["launches"],
                    "algo_bytes_per_launch": dom["algo_bytes_per_launch"],
                    "timing": "HIP events around every full-work launch of every 8th solve of the timed steps",
                    "other": other}

    variants = None
    if a.variant_steps > 0:
        variants = run_variants(S, w, prob, stream, ud, dt, a.variant_steps, dof_updates, start)

    cpu = None
    if not a.no_cpu_baseline:
        if w["eq"] == "ns":
            cpu = ns_cpu_baseline(S, w, prob, meth, stream, dev, nsteps=a.cpu_steps)
        else:
            Ei = E // B  # a stacked ensemble: the oracle steps its first instance
            with tempfile.TemporaryDirectory() as td:
                p0 = os.path.join(td, "u0.npy")
                p1 = os.path.join(td, "g1.npy")
                np.save(p0, u0[:, :Ei])
                np.save(p1, step1.reshape(nv, E, Np)[:, :Ei])
                r = cpu_baseline(w, p0, p1, a.cpu_steps)
            cpu_rate = dof_updates / B * r["steps"] / r["seconds"]
            cpu = {"value": cpu_rate, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
                   "sample": f"{r['steps']} time steps of the same workload from the same u0 "
                             + (f"(its first instance) " if B > 1 else "")
                             + f"(oracle CG to the same 1e-10 tolerance), {r['seconds']:.1f} s",
                   "gpu_vs_oracle_rel_l2_step1": r["rel_l2_step1"]}

    single = None
    if B > 1:  # the ensemble's first instance stepped alone, for comparison
        single = single_instance_rate(S, w, prob, meth, u0[:, :E // B], dt, a.steps, a.warmup,
                                      dof_updates / B, stream)
    rec = {
        "metric": "fine-level DOF-updates/s (s/step at fixed PCG tolerance 1e-10)",
        "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded Fourier initial data)",
        "config": {"workload": w["name"], "levels_P": w["P"], "levels_M": w["M"], "global_batch": B, "seq_len": None, "parallelism": "none",
                   "single_instance": single, "ms_per_step_median": ms_median,
                   "rel_l2_error_vs_exact_solution": err_exact,
                   "dt": dt, "fine_dof": E * Np * nv, "fine_sweeps_per_step": sweeps,
                   "cg_iters_per_step": tot["cg_iters"] / a.steps, "solves_per_step": tot["solves"] / a.steps,
                   "not_converged": tot["not_converged"], "max_rel_residual": tot["max_rel_residual"],
                   "wall_s": wall},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(rec), flush=True)
    sv.close()


if __name__ == "__main__":
    main()
