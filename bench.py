"""Benchmark of the DGSEM hot path on one MI355X.

Default workload: Taylor-Green vortex (Re 1600, Ma 0.1, Version II) on a curved
periodic 24^3 hexahedral mesh, N = 7 Gauss nodes (7,077,888 DOF), Roe + BR1,
LSERK4-5, FP64.  A step is one RK step: five evaluations of the whole operator
(traces, BR1 lifting, face fluxes, volume and surface integrals, Jacobian)
and the stage updates.  value = DOF * 5 * steps / wall time (DOF counts
nodes, as the paper's PID does); PID = 1 / value at one GPU.

Also reported on the same line: the per-kernel roofline of the dominant
kernel (HIP events on the solver's stream), the mixed-precision form on the
32^3 mesh, the p50/p99 latency of whole solves, and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64, vector or matrix


def algorithmic_bytes_per_dof(N: int, mixed: bool):
    """minimum HBM bytes per DOF and stage of the two sweeps of the viscous
    operator (BR1 needs every neighbour's lifted gradient before a viscous face
    flux exists).  Volume sweep: reads U, Ja, 1/J and the neighbours' U traces;
    writes each own face node's viscous normal flux (4 values) and the volume
    integral (5).  Surface sweep: reads U, du, the volume integral, 1/J, the
    neighbours' U traces and both sides' viscous face fluxes; writes du, U and
    the next U traces.  An element's own U traces follow from its U and are not
    counted, nor are the face normals.  f = 6/(N+1) face slots per DOF."""
    f = 6.0 / (N + 1)
    if not mixed:
        vol = 8 * (20 + 9 * f)
        surf = 8 * (26 + 18 * f)
    else:  # U and du in FP64; metrics, traces, face fluxes, volume integral in FP32
        vol = 8 * 5 + 4 * (15 + 9 * f)
        surf = 8 * 20 + 4 * (6 + 18 * f)
    return vol, surf


# the paper's memory per DOF of its Navier-Stokes solver (Sec. 4.3, Table
# tab:memory_requirements), KiB per DOF at N = 3, 5, 7 on its GPUs
PAPER_KIB_PER_DOF = {3: 1.049, 5: 0.942, 7: 0.869}


def memory_per_dof(P, W):
    """device workspace bytes per DOF of one solve, per degree and form"""
    out = []
    for N in range(1, 10):
        E = 4096
        dof = E * (N + 1) ** 3
        row = {"N": N}
        for name, prm in (("fp64", W.params(N, riemann=1)), ("mixed", W.params(N, riemann=1, precision=1)),
                          ("split_fp64", W.params(N, node_type=1, volume_flux=1)),
                          ("ctgv_fp64", W.params(N, node_type=1, volume_flux=1, shock=1, viscosity=1)
                           if 2 <= N <= 7 else None)):
            if prm is None:
                continue
            row[name + "_B_per_dof"] = P.workspace_bytes(prm, E) / dof
        if N in PAPER_KIB_PER_DOF:
            row["paper_B_per_dof"] = PAPER_KIB_PER_DOF[N] * 1024
        out.append(row)
    return out


def pid_sweep(P, W, Ks, steps, split):
    """PID (s) against DOF on one GPU at N = 7 (Sec. 4.4, the one-GPU part of
    the scaling figure): curved TGV boxes of K^3 elements; standard form on
    Gauss nodes, or the split form on Gauss-Lobatto nodes"""
    import torch
    rows = []
    for K in Ks:
        # Cartesian boxes (geometry on the element corners): the cost per DOF
        # does not depend on the curving, which only the metric values carry
        if split:
            wl = W.compressible_tgv_workload(K=K, N=7, curved=False, ngeo=1)
            wl.params = dict(wl.params, shock_capturing=0, time_scheme=0)
        else:
            wl = W.tgv_workload(K=K, N=7, curved=False, ngeo=1)
        s = P.Solver(wl.params, wl.mesh)
        s.set_state(wl.U0, 0.0)
        dt = s.stable_dt(0.5, 0.5)
        s.advance(2, dt)
        s.synchronize()
        n = max(2, min(steps, int(4e9 / (wl.dof * 5))))  # about half a second of work
        t0 = time.perf_counter()
        s.advance(n, dt)
        s.synchronize()
        el = time.perf_counter() - t0
        rows.append({"K": K, "dof": wl.dof, "steps": n, "pid_s": el / (wl.dof * 5 * n),
                     "value": wl.dof * 5 * n / el})
        progress(f"  PID sweep {'split' if split else 'standard'} K={K}: {rows[-1]['pid_s']:.3e} s")
        del s
        torch.cuda.empty_cache()
    return rows


_T0 = time.perf_counter()


def progress(msg):
    """a progress line on stderr (stdout carries the one JSON result line),
    with the seconds since the start"""
    print(f"[bench {time.perf_counter() - _T0:6.1f} s] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2404_12703_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(name):
    """a committed rocprofv3 counter record (HBM bytes per launch from
    FETCH_SIZE/WRITE_SIZE, or FP64 VALU flops per launch from SQ counters),
    valid only for the kernel sources it was taken on"""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def time_solver(P, wl, steps, warmup, profile_pass=True):
    import torch
    s = P.Solver(wl.params, wl.mesh)
    s.set_state(wl.U0, 0.0)
    dt = s.stable_dt(0.9, 0.9)
    s.advance(warmup, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(steps, dt)
    s.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = None
    if profile_pass:
        s.profile(True)
        s.advance(steps, dt)
        prof = s.profile_read()
        s.profile(False)
    return s, dt, el, prof


def solve_latency(P, wl, steps, repeats, cfl=None, dt=None):
    """`repeats` full solves (set_state from a device copy, `steps` RK steps,
    state read back into device memory), each timed on the host clock, after
    one untimed solve (the first launch of each kernel loads its code object).
    Returns p50/p99 and the solver, holding the last solve's final state."""
    import torch
    s = P.Solver(wl.params, wl.mesh)
    s.set_state(wl.U0, 0.0)
    if dt is None:
        c = wl.cfl if cfl is None else cfl
        dt = s.stable_dt(c, c)
    U0 = torch.from_numpy(wl.U0).cuda()
    out = torch.empty_like(U0)
    lat = []
    for rep in range(repeats + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_state(U0, 0.0)
        s.advance(steps, dt)
        s.state_into(out)
        s.synchronize()
        if rep:
            lat.append(time.perf_counter() - t0)
    st = {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)), "repeats": repeats,
          "steps": steps, "dt": dt, "solve": f"set_state + {steps} steps + get_state",
          "value_at_p50": wl.dof * 5 * steps / float(np.percentile(lat, 50))}
    return st, s, out


_STREAMS = {}
MAX_ACTIVE = 128  # requests the server runs together (--max-active)


def stream_workloads(W, nreq, seed, precision):
    """the served stream's requests as workloads (built once per precision)"""
    key = (nreq, seed, precision)
    if key not in _STREAMS:
        base = W.serving_requests(nreq, seed, rate=1.0)
        _STREAMS[key] = (base, [W.request_workload(r, precision=precision) for r in base])
    return _STREAMS[key]


def served(P, W, nreq, seed, throughput, load=0.8, precision=0, budget=32 << 30, max_active=None):
    """the served stream: nreq seeded requests (K in 4..16, N in {3,5,7},
    Ma, Re, steps drawn per request) with Poisson arrivals at `load` times the
    measured throughput (load None: all at t = 0), FIFO admission under an
    HBM budget.  Returns throughput over the makespan and p50/p99 of
    t_done - t_arrival."""
    import torch
    base, wls = stream_workloads(W, nreq, seed, precision)
    work = [(r["K"] ** 3) * (r["N"] + 1) ** 3 * 5 * r["steps"] for r in base]
    if load is None:  # every request arrives at t = 0
        arrivals = np.zeros(nreq)
    else:
        lam = load * throughput / float(np.mean(work))
        g = np.random.default_rng(seed + 1000)
        arrivals = np.cumsum(g.exponential(1.0 / lam, size=nreq))
    if max_active is None:
        max_active = MAX_ACTIVE
    arena = min(budget + (256 << 20), int(torch.cuda.mem_get_info()[0] * 0.8))
    sv = P.Server(arena_bytes=arena, hbm_budget=budget, max_active=max_active)
    # the whole stream is submitted before the loop starts; arrival times are
    # on the server clock, which starts with the loop
    ids = []
    for i, (r, wl, ta) in enumerate(zip(base, wls, arrivals)):
        ids.append(sv.submit(wl.params, wl.mesh, wl.U0, r["steps"], -0.9, float(ta)))
        if (i + 1) % 128 == 0:
            progress(f"  submitted {i + 1}/{nreq}")
    t0 = time.perf_counter()
    sv.run(0)
    makespan = time.perf_counter() - t0
    progress(f"served {nreq} requests, load {load}, precision {precision}: {makespan:.1f} s")
    lat, ok = [], 0
    for rid in ids:
        _, tm = sv.fetch(rid)
        ok += tm["state"] == P.REQ_DONE
        lat.append(tm["t_done"] - tm["t_arrival"])
    stats = sv.stats()
    sv.close()
    return dict(stats=stats, requests=nreq, done=ok, load=("all at t=0" if load is None else load), precision=precision,
                value=float(np.sum(work)) / makespan, unit="DOF*stage/s",
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                makespan_s=makespan, budget_GB=budget / 2 ** 30)


_ONE_THREAD = """
import sys, time
sys.path.insert(0, {root!r})
import oracle as O, workloads as W
wl = W.tgv_workload(K={K}, N=7, steps=1)
o = O.Oracle(wl.params, wl.mesh)
t0 = time.perf_counter()
o.rhs(wl.U0)
print(time.perf_counter() - t0)
"""


def cpu_baseline(wl, K, seconds_budget=30.0):
    """the FP64 oracle, untuned, on the host cores: one full RK step (five
    operator evaluations) of the same workload; and on one thread (a child
    process, since the thread count is fixed when the oracle loads) one
    operator evaluation"""
    import subprocess
    import oracle as O
    o = O.Oracle(wl.params, wl.mesh)
    dt = o.stable_dt(wl.U0)
    t0 = time.perf_counter()
    o.advance(wl.U0, dt, 1)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = dict(value=wl.dof * 5 / el, unit="DOF*stage/s", cores=cores, kind="oracle",
               sample=f"1 RK step (5 operator evaluations) of the full {wl.name} workload, {el:.1f} s")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", _ONE_THREAD.format(root=ROOT, K=K)], env=env, capture_output=True,
                           text=True, timeout=10 * seconds_budget)
        el1 = float(r.stdout.strip().splitlines()[-1])
        out["one_thread"] = dict(value=wl.dof / el1, unit="DOF*stage/s", cores=1,
                                 sample=f"1 operator evaluation of the full {wl.name} workload, {el1:.1f} s")
    except Exception as ex:  # reported, not fatal: the baseline is context
        out["one_thread"] = dict(value=None, error=str(ex)[:200])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--K", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serve-requests", type=int, default=512, help="requests of the served stream")
    ap.add_argument("--no-extras", action="store_true", help="skip mixed precision and latency")
    ap.add_argument("--only-main", action="store_true", help="time the main workload only (profiling runs)")
    ap.add_argument("--only-blast", action="store_true",
                    help="time the shock-capturing blast workload only (profiling runs of that path)")
    ap.add_argument("--only-ctgv", action="store_true",
                    help="time the supersonic split-form TGV only (profiling runs of that path)")
    ap.add_argument("--only-served", action="store_true",
                    help="the served stream only (FP64, load 0.8 and all at t = 0), with the loop statistics")
    ap.add_argument("--only-mixed", action="store_true",
                    help="time the mixed-precision 32^3 TGV only (profiling runs of that path)")
    ap.add_argument("--max-active", type=int, default=128, help="requests the server runs together")
    ap.add_argument("--full", action="store_true",
                    help="every section at full size (about 7 minutes): the served stream at four FP64 loads "
                         "and two mixed, the PID sweep to 1e8 DOF, five solves per mixed-precision latency")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain 1 GiB read + 1 GiB write elementwise kernel (counter calibration)")
    args = ap.parse_args()
    global MAX_ACTIVE
    MAX_ACTIVE = args.max_active
    if args.gpus != 1:
        print("bench.py: measures one GPU (--gpus 1); the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2404_12703_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calib:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        copy_gbs = 10 * 2 * (1 << 30) / (time.perf_counter() - t0) / 1e9
        del a, b
    if args.only_blast:
        wb = W.blast_workload(K=32, N=5)
        sbl = P.Solver(wb.params, wb.mesh)
        sbl.set_state(wb.U0, 0.0)
        dtb = sbl.stable_dt(wb.cfl, wb.cfl)
        sbl.advance(args.warmup, dtb)
        sbl.synchronize()
        t0 = time.perf_counter()
        sbl.advance(args.steps, dtb)
        sbl.synchronize()
        elb = time.perf_counter() - t0
        sbl.profile(True)
        sbl.advance(args.steps, dtb)
        pb = sbl.profile_read()
        sbl.profile(False)
        print(json.dumps({"workload": "blast 32^3 N=5 Lobatto, indicator + FV blend, FP64", "steps": args.steps,
                          "value": wb.dof * 5 * args.steps / elb, "unit": "DOF*stage/s",
                          "k_volume_ms": pb["lift"][0] / pb["lift"][1], "k_surface_ms": pb["rhs"][0] / pb["rhs"][1],
                          "alpha_pos_fraction": float(np.mean(sbl.alpha() > 0))}), flush=True)
        return
    if args.only_ctgv:
        wc = W.compressible_tgv_workload(K=args.K, N=7, curved=True)
        sc = P.Solver(wc.params, wc.mesh)
        sc.set_state(wc.U0, 0.0)
        dtc = sc.stable_dt(wc.cfl, wc.cfl)
        sc.advance(args.warmup, dtc)
        sc.synchronize()
        t0 = time.perf_counter()
        sc.advance(args.steps, dtc)
        sc.synchronize()
        elc = time.perf_counter() - t0
        print(json.dumps({"workload": "supersonic TGV 24^3 N=7 Lobatto, split form, 14-stage RK, FP64",
                          "steps": args.steps, "value": wc.dof * 14 * args.steps / elc, "unit": "DOF*stage/s",
                          "alpha_pos_fraction": float(np.mean(sc.alpha() > 0))}), flush=True)
        return
    if args.only_mixed:
        wm = W.tgv_workload(K=32, N=7, precision=1)
        s, dt, el, prof = time_solver(P, wm, args.steps, args.warmup, profile_pass=True)
        vbm, sbm = algorithmic_bytes_per_dof(7, True)
        out = {"workload": "tgv 32^3 N=7 mixed precision (p_ref = p0)", "steps": args.steps,
               "value": wm.dof * 5 * args.steps / el, "unit": "DOF*stage/s"}
        for key, name, b in (("lift", "k_volume", vbm), ("rhs", "k_surface", sbm)):
            t = prof[key][0] / prof[key][1] * 1e-3
            out[name] = {"avg_ms": t * 1e3, "alg_bytes_per_dof": b, "frac": b * wm.dof / t / 1e9 / HBM_PEAK_GBS}
        print(json.dumps(out), flush=True)
        return
    if args.only_served:
        wl = W.tgv_workload(K=args.K, N=7, steps=10)
        _, _, el, _ = time_solver(P, wl, 10, 2, profile_pass=False)
        rate = wl.dof * 5 * 10 / el
        out = {"single_solve_value": rate,
               "served": [served(P, W, args.serve_requests, 0, rate, load=ld, precision=0) for ld in (None, 0.8)]}
        print(json.dumps(out), flush=True)
        return
    wl = W.tgv_workload(K=args.K, N=7, steps=args.steps)
    N = 7
    progress(f"main workload: {wl.dof} DOF, {args.steps} steps")
    s, dt, el, prof = time_solver(P, wl, args.steps, args.warmup, profile_pass=not args.only_main)
    value = wl.dof * 5 * args.steps / el
    line = {
        "metric": "DOF*RK-stage updates/s (PID = 1/value) FP64 on 1 GPU; p50/p99 solve latency",
        "value": value, "unit": "DOF*stage/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"tgv_re1600_ma0.1_curved_{args.K}^3_N7_gauss_roe_br1_lserk45_fp64",
                   "elements": wl.mesh.n_elems, "N": N, "dof": wl.dof, "dt": dt},
        "pid_s": 1.0 / value,
    }
    if args.copy_calib:
        line["copy_kernel_GBs"] = copy_gbs
    if not args.only_main:
        # the same timed interval four more times: median and spread of five
        import torch
        vals = [value]
        for _ in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.advance(args.steps, dt)
            s.synchronize()
            torch.cuda.synchronize()
            vals.append(wl.dof * 5 * args.steps / (time.perf_counter() - t0))
        line["repeats"] = {"n": 5, "median": float(np.median(vals)), "min": float(np.min(vals)),
                           "max": float(np.max(vals))}
    if prof is not None:
        vol_b, surf_b = algorithmic_bytes_per_dof(N, False)
        names = {"lift": ("k_volume", "Lift_* + VolInt + own-side viscous face flux", vol_b),
                 "rhs": ("k_surface", "FillFlux + SurfInt + ApplyJac + LSERK update + ProlongToFace", surf_b)}
        tr = load_traffic("traffic_tgv24_n7_fp64.json")
        va = load_traffic("valu_tgv24_n7_fp64.json")  # FP64 VALU flops per launch from SQ counters
        kern = {}
        for key, (name, what, b) in names.items():
            ms, nl = prof[key]
            t = ms / nl * 1e-3
            kern[name] = {"computes": what, "avg_ms": t * 1e3, "launches": nl, "alg_bytes_per_dof": b,
                          "alg_GBs": b * wl.dof / t / 1e9,
                          "traffic_bytes_per_launch": (tr["kernels"][name] if tr else None)}
            if va:
                fl = va["kernels"][name]["fp64_flop_per_launch"]
                kern[name].update(fp64_flop_per_launch=fl, fp64_TFLOPs=fl / t / 1e12,
                                  fp64_frac=fl / t / 1e12 / FP64_PEAK_TFLOPS,
                                  mfma_instr=va["kernels"][name]["mfma_f64_instr"],
                                  lds_idx_active=va["kernels"][name]["lds_idx_active_per_busy_cycle"])
        dom = max(kern, key=lambda k: kern[k]["avg_ms"])
        kd = kern[dom]
        line["roofline"] = {"kernel": f"{dom} ({kd['computes']})", "bound": "hbm", "achieved": kd["alg_GBs"],
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kd["alg_GBs"] / HBM_PEAK_GBS,
                            "traffic": kd["traffic_bytes_per_launch"],
                            "alg_bytes_per_launch": kd["alg_bytes_per_dof"] * wl.dof,
                            "avg_launch_ms": kd["avg_ms"]}
        if va and kd.get("lds_idx_active") is not None:
            # what holds the dominant kernel below the HBM roofline, from the
            # committed SQ counter record of the same kernel sources
            lim = (f"LDS: its index unit is active in {kd['lds_idx_active']:.2f} of the CU-busy cycles while FP64 "
                   f"arithmetic runs at {kd['fp64_frac']:.2f} of peak")
            if kd["traffic_bytes_per_launch"]:
                lim += f" and measured HBM traffic at {kd['traffic_bytes_per_launch'] / (kd['avg_ms'] * 1e6):.0f} GB/s"
            line["roofline"]["limiter"] = lim
        line["kernels"] = kern
        # the counter-derived fields above come from committed records, used
        # only while the kernel sources hash to the value they were taken on
        line["counter_records"] = {"kernel_source_hash": kernel_source_hash(),
                                   "traffic": "profiles/traffic_tgv24_n7_fp64.json" if tr else None,
                                   "valu_lds": "profiles/valu_tgv24_n7_fp64.json" if va else None}
        step_alg = (vol_b + surf_b) * wl.dof * 5 * args.steps / el / 1e9
        line["whole_step_alg_GBs"] = step_alg
        line["whole_step_hbm_frac"] = step_alg / HBM_PEAK_GBS
    del s
    torch.cuda.empty_cache()
    if not args.no_extras and not args.only_main:
        # mixed precision against FP64 on the 32^3 mesh: 500 steps with the same dt,
        # five full solves each; E_k and the state of the last solves compared
        nmix = 5 if args.full else 3
        progress(f"mixed precision against FP64, 32^3, 500 steps x {nmix} solves each")
        wd = W.tgv_workload(K=32, N=7, precision=0)
        wm = W.tgv_workload(K=32, N=7, precision=1)
        std, sd, Ud = solve_latency(P, wd, 500, nmix)
        stm, sm, Um = solve_latency(P, wm, 500, nmix, dt=std["dt"])
        Id, Im = sd.integrals(), sm.integrals()
        # per-kernel times of the mixed form (HIP events on its stream)
        sm.profile(True)
        sm.advance(10, std["dt"])
        pm = sm.profile_read()
        sm.profile(False)
        vbm, sbm = algorithmic_bytes_per_dof(7, True)
        mixed_k = {}
        for key, name, b in (("lift", "k_volume", vbm), ("rhs", "k_surface", sbm)):
            t = pm[key][0] / pm[key][1] * 1e-3
            mixed_k[name] = {"avg_ms": t * 1e3, "alg_bytes_per_dof": b, "alg_GBs": b * wm.dof / t / 1e9,
                             "frac": b * wm.dof / t / 1e9 / HBM_PEAK_GBS}
        line["mixed_tgv32"] = {
            "dof": wd.dof, "steps": 500, "fp64": std, "mixed": stm,
            "speedup": std["p50_s"] / stm["p50_s"],
            "kernels": mixed_k,
            "ek_rel_err": abs(Im[5] - Id[5]) / abs(Id[5]),
            "state_rel_l2": float(torch.linalg.norm(Um - Ud) / torch.linalg.norm(Ud))}
        del sd, sm, Ud, Um
        torch.cuda.empty_cache()
        progress("latency of whole solves")
        st, s2, _ = solve_latency(P, W.tgv_workload(K=args.K, N=7), args.steps, 20)
        line["latency_tgv24"] = st
        del s2
        st, s1, _ = solve_latency(P, W.mms_workload(), 10, 20)
        line["latency_mms"] = st
        del s1
        # the shock-capturing workload: 32^3 Lobatto N=5, indicator + FV blend
        progress("blast 32^3, 200 steps x 5 solves")
        wb = W.blast_workload(K=32, N=5)
        st, sbl, _ = solve_latency(P, wb, 200, 5)
        sbl.set_state(wb.U0, 0.0)
        sbl.rhs(0.0)
        st["alpha_pos_fraction_t0"] = float(np.mean(sbl.alpha() > 0))
        line["blast32"] = st
        del sbl
        torch.cuda.empty_cache()
        # the supersonic Taylor-Green vortex: split form (Pirozzoli), Sutherland,
        # indicator + FV blend, fourteen-stage RK; 24^3 curved, N = 7 Lobatto
        progress("supersonic split-form TGV")
        wc = W.compressible_tgv_workload(K=args.K, N=7, curved=True)
        sc = P.Solver(wc.params, wc.mesh)
        sc.set_state(wc.U0, 0.0)
        dtc = sc.stable_dt(wc.cfl, wc.cfl)
        sc.advance(2, dtc)
        sc.synchronize()
        nst = 20
        t0 = time.perf_counter()
        sc.advance(nst, dtc)
        sc.synchronize()
        elc = time.perf_counter() - t0
        sc.profile(True)
        sc.advance(2, dtc)
        pc = sc.profile_read()
        sc.profile(False)
        line["ctgv24_split"] = {
            "workload": "supersonic TGV Ma 1.25 Re 1600, curved 24^3, N=7 Lobatto, split form + Sutherland + "
                        "indicator/FV blend + 14-stage RK, FP64",
            "dof": wc.dof, "steps": nst, "stages_per_step": 14, "dt": dtc,
            "value": wc.dof * 14 * nst / elc, "unit": "DOF*stage/s", "pid_s": elc / (wc.dof * 14 * nst),
            "k_volume_ms": pc["lift"][0] / pc["lift"][1], "k_surface_ms": pc["rhs"][0] / pc["rhs"][1],
            "alpha_pos_fraction": float(np.mean(sc.alpha() > 0)),
            "eps_S_eps_D": [float(x) for x in sc.dissipation()], "finite": bool(np.isfinite(sc.integrals()).all())}
        del sc
        torch.cuda.empty_cache()
        # its evolution on 16^3 elements to t = 11 (shocks from t ~ 1.7): the
        # quantities of the paper's compressible TGV figure, without its
        # reference data
        progress("supersonic TGV evolution, 16^3")
        we = W.compressible_tgv_workload(K=16, N=7, curved=False)
        se = P.Solver(we.params, we.mesh)
        se.set_state(we.U0, 0.0)
        dte = se.stable_dt(we.cfl, we.cfl)
        evo = []
        for blk in range(10):
            se.advance(250, dte)
            I, eps = se.integrals(), se.dissipation()
            evo.append({"t": 250 * (blk + 1) * dte, "E_k": float(I[5]), "eps_S": float(eps[0]),
                        "eps_D": float(eps[1]), "blended_fraction": float(np.mean(se.alpha() > 0))})
        line["ctgv16_evolution"] = {"dof": we.dof, "dt": dte, "samples": evo}
        del se
        torch.cuda.empty_cache()
        # the served stream: at the arrival ceiling (load 0.8) and saturated
        # (all at t = 0); --full adds loads 0.5 and 1.2 in FP64 and 0.8 mixed
        loads64 = (0.5, 0.8, 1.2, None) if args.full else (0.8, None)
        loads32 = (0.8, None) if args.full else (None,)
        line["served"] = [served(P, W, args.serve_requests, 0, value, load=ld, precision=0) for ld in loads64]
        line["served"] += [served(P, W, args.serve_requests, 0, value, load=ld, precision=1) for ld in loads32]
        progress("PID sweep")
        # to 1.7e7 DOF by default (the PID is flat above 1e6); --full to 1e8
        ks = (3, 4, 6, 8, 12, 16, 24, 32, 48, 58) if args.full else (3, 4, 6, 8, 12, 16, 24, 32)
        kss = (3, 4, 6, 8, 12, 16, 24, 32, 48) if args.full else (3, 6, 12, 24)
        line["pid_sweep_n7"] = {"standard_gauss": pid_sweep(P, W, ks, 20, split=False),
                                "split_lobatto": pid_sweep(P, W, kss, 20, split=True)}
        line["bench_sections"] = "full" if args.full else "default (bench.py --full for every load and size)"
        line["memory_per_dof"] = memory_per_dof(P, W)
    if not args.no_cpu and not args.only_main:
        progress("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(W.tgv_workload(K=args.K, N=7, steps=1), args.K)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
