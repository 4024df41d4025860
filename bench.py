#!/usr/bin/env python3
"""Benchmark of one full IB-LB step on one MI355X.

Workload (default, ``--workload wetting128``): the 128x128x96 wetting droplet
-- no-slip walls at z = 0 and 95, a softly coated droplet alpha = abar(1,0,1),
abar = 1e-4, meshed as a level-5 icosphere (10242 vertices, 20480 faces, R =
24), a wetting lower wall (eps/abar = 1, r_cut = 2) -- with FP32 deviation
populations and FP64 positions and volume reductions.  Synthetic seeded
inputs, no datasets.

Timed region: W untimed warm-up steps, then exactly K steps replayed from
hipGraphs captured before the warm-up (16-step graphs, one-step graphs for the
remainder, either start parity), inputs resident in HBM.  hipEvents on the
library's stream bracket the K steps, inside torch.cuda.synchronize() on both
sides.  value = fluid nodes x K / event seconds / 1e6 (MLUPS) for the whole
step (forces, spreading, LB, moments, interpolation and move).

roofline: the whole step as one unit of work.  achieved = the step's
algorithmic bytes (the LB's 38 population accesses per fluid node plus the
interface terms on the shell nodes, faces and vertices) / the event-timed step;
peak = 8 TB/s HBM.  traffic = HBM bytes per step from committed
FETCH_SIZE/WRITE_SIZE counter runs over the four dispatches of a step
(copy-calibrated), while the kernel source is the one they were taken on, else
null.  "dispatches" breaks the step into its four dispatches, timed one by one
with hipEvents in a separate pass of plain launches, each with its own share of
the algorithmic bytes.  Secondary figures: the LB kernel alone on the same
lattice without a mesh ("lb_only"), the 256^3 probe beyond the Infinity Cache
("probe256"), and a plain device copy ("device_copy").  "adjoint": the
adjoint/forward time ratio of the differentiation workload (64x64x48, 2000
steps, checkpoints every 100) with the largest relative error of its gradients
against central finite differences.  The FP64 CPU oracle is timed on a bounded
sample of the same workload on all host cores and on one.

--pass lb / --pass copy run only the LB-only pass, or a plain device copy of
--copy-mib MiB, for hardware-counter runs.  --study precision runs the
contact-angle comparison of the population storage precisions instead,
--study shear the capillary-number sweep of the sheared particles, and
--study batch the 48-domain parameter sweep stepped as one batch against the
same domains stepped one at a time, and --study adjoint the gradient of the
wetting observables by the adjoint, its cost relative to the forward run and
its error against finite differences, and --study wetting the equilibrium
contact angle against the wall strength for the pre-stressed models.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline per IB-LB step; adjoint/forward time ratio at stated accuracy"
HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 * 2**20  # MI355X last-level (MALL) cache
DISPATCHES = ("forces", "spread", "moments", "move")


def workload(name: str):
    from paper_2305_18919_amd import inputs as I
    if name == "shear64":
        return I.c2_shear(0.05), 1
    if name == "droplet32":
        return I.c1_droplet(), 0
    if name == "wetting128":
        return I.c3_wetting(1.0), 1
    if name == "probe256":
        return probe256(), 1
    raise SystemExit(f"unknown workload {name}")


def probe256():
    """The wetting droplet of the 128x128x96 case in a 256^3 lattice: 1.26 GB of
    FP32 populations, far beyond the 256 MB Infinity Cache."""
    from paper_2305_18919_amd import inputs as I
    w = I.c3_wetting(1.0)
    w.domain = I.Domain(256, 256, 256)
    w.mesh.vertices = w.mesh.vertices + [64.0, 64.0, 0.0]
    w.mesh.ref_vertices = w.mesh.ref_vertices + [64.0, 64.0, 0.0]
    w.name = "probe256_f32"
    return w


POP_BYTES = {0: 8, 1: 4, 2: 2, 3: 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
DTYPE = {0: "f64", 1: "f32", 2: "f16 storage, f32 arithmetic", 3: "bf16 storage, f32 arithmetic"}


def lb_bytes_per_node(precision: int) -> int:
    return 38 * POP_BYTES[precision]


# ----------------------------------------------------------------- host bookkeeping

def step_geometry(dom, q, split: dict, tile=None) -> dict:
    """Node counts behind the algorithmic bytes of one step at positions q.

    shell: fluid nodes inside some vertex's 4^3 stencil; active: nodes of the
    tiles (extents `tile`, the library's by default) those stencils reach (the
    spreading dispatch updates them).  Per
    dispatch, the LB nodes it updates: the LB blocks of the other nodes (block
    width and forces share of the library's split) go first to the forces
    dispatch, the rest to the spreading dispatch."""
    import numpy as np
    if tile is None:
        from paper_2305_18919_amd import iblb
        tile = iblb.tile_shape()
    tx, ty, tz = tile
    nx, ny, nzf = dom.nx, dom.ny, dom.nz_fluid
    walls = dom.wall_mode == 0
    b = np.floor(q).astype(np.int64) - 1
    k = np.arange(4)
    xs = (b[:, 0, None] + k) % nx
    ys = (b[:, 1, None] + k) % ny
    zs = b[:, 2, None] + k - (1 if walls else 0)
    if not walls:
        zs = zs % nzf
    X = np.broadcast_to(xs[:, None, None, :], (len(q), 4, 4, 4))
    Y = np.broadcast_to(ys[:, None, :, None], (len(q), 4, 4, 4))
    Z = np.broadcast_to(zs[:, :, None, None], (len(q), 4, 4, 4))
    ok = (Z >= 0) & (Z < nzf)
    shell = np.zeros((nzf, ny, nx), dtype=bool)
    shell[Z[ok], Y[ok], X[ok]] = True
    ntz, nty, ntx = -(-nzf // tz), -(-ny // ty), -(-nx // tx)
    tiles = np.zeros((ntz, nty, ntx), dtype=bool)
    tiles[Z[ok] // tz, Y[ok] // ty, X[ok] // tx] = True
    act = tiles[(np.arange(nzf) // tz)[:, None, None], (np.arange(ny) // ty)[None, :, None],
                (np.arange(nx) // tx)[None, None, :]]
    bxw = split["block_x"]
    byw = 256 // bxw
    nbx, nby = (nx + bxw - 1) // bxw, (ny + byw - 1) // byw
    pad = ((0, 0), (0, nby * byw - ny), (0, nbx * bxw - nx))
    other = (~np.pad(act, pad, constant_values=True)).reshape(nzf, nby, byw, nbx, bxw).sum(axis=(2, 4)).reshape(-1)
    nb = other.size
    e0 = int(split["share_forces"] * nb + 0.5)
    n_act = int(act.sum())
    lb = {"forces": int(other[:e0].sum()), "spread": int(other[e0:].sum()) + n_act, "moments": 0, "move": 0}
    assert sum(lb.values()) == dom.n_fluid, (lb, dom.n_fluid)
    return {"shell_nodes": int(shell.sum()), "active_nodes": n_act, "lb_nodes": lb, "lb_blocks": nb}


def algorithmic_bytes(dom, mesh, prec: int, geo: dict) -> dict:
    """Bytes the method must move in one step, per dispatch: every fluid node's
    19 populations read and written once (38 s_pop), the shell nodes' force
    density written and read (6 s_F), their populations read again and u(t+1)
    written and read for the interpolation (19 s_pop + 8 s_F), the faces'
    indices, reference data and corner force and volume terms (12 + 40 s_F),
    and the vertices' FP64 positions, nodal forces and incidence (104 + 6 s_F +
    48 B).  s_pop: bytes per stored population; s_F: bytes per value of the
    step's arithmetic type."""
    sp, sf = POP_BYTES[prec], (8 if prec == 0 else 4)
    ns, nf, nv = geo["shell_nodes"], mesh.n_faces, mesh.n_vertices
    lb = {k: v * 38 * sp for k, v in geo["lb_nodes"].items()}
    ib = {
        "forces": nf * (12 + 4 * sf + 36 * sf) + nv * (48 + 8) + 6 * nv * 8,
        "spread": ns * 6 * sf + nv * 6 * sf,
        "moments": ns * (19 * sp + 4 * sf),
        "move": ns * 4 * sf + nv * 48,
    }
    per = {k: lb[k] + ib[k] for k in DISPATCHES}
    return {"total": sum(per.values()), "lb": sum(lb.values()), "ib": sum(ib.values()), "per_dispatch": per}


# ----------------------------------------------------------------- GPU timing

def event_time(stream, fn):
    """Milliseconds between hipEvents recorded on `stream` around fn()."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def step_traffic(workload_name: str, prec: int):
    """HBM bytes per step (the four dispatches) from the committed
    FETCH_SIZE/WRITE_SIZE runs (copy-calibrated), or None when they were
    taken on another kernel source or another workload."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "step_wetting128_f32_counters.json")
    if workload_name != "wetting128_f32" or prec != 1 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return int(rec["traffic_bytes_per_step"])


def lb_roofline(dom, prec: int, launches: int):
    """k_lb over every fluid node of the domain (no mesh), graph-replayed;
    hipEvents on the library stream around `launches` consecutive launches."""
    from paper_2305_18919_amd import iblb
    launches = max(16, launches // 16 * 16)
    with iblb.Simulation(dom, None, precision=prec, graph=True) as sim:
        sim.step(64)
        sim.sync()
        ms = event_time(sim.stream, lambda: sim.step(launches))
        sim.sync()
    us = ms * 1e3 / launches
    alg = dom.n_fluid * lb_bytes_per_node(prec)
    achieved = alg / (us * 1e-6) / 1e9
    out = {"kernel": "k_lb (every fluid node, no mesh)", "fluid_nodes": dom.n_fluid, "alg_bytes_per_launch": alg,
           "launches": launches, "avg_us": round(us, 3), "achieved_GBs": round(achieved, 1),
           "frac": round(achieved / HBM_PEAK_GBS, 4)}
    if alg / 2 < INFINITY_CACHE_BYTES:
        # the populations (half the bytes moved) fit in the MI355X's last-level
        # cache and stay there between launches: the rate is not HBM's
        out["note"] = "populations resident in the 256 MB Infinity Cache; the 256^3 probe is the HBM-bound case"
    return out


def coupled_rate(w, prec: int, steps: int, warmup: int):
    """Graph-replayed coupled steps of workload w: (us per step, MLUPS, the
    step's algorithmic bytes at the positions after the timed steps)."""
    import numpy as np
    from paper_2305_18919_amd import iblb
    with iblb.Simulation(w.domain, w.mesh, precision=prec, graph=True) as sim:
        sim.step(warmup)
        sim.sync()
        ms = event_time(sim.stream, lambda: sim.step(steps))
        sim.sync()
        split = sim.lb_split()
        q = np.asarray(sim.vertices())
    us = ms * 1e3 / steps
    alg = algorithmic_bytes(w.domain, w.mesh, prec, step_geometry(w.domain, q, split))["total"]
    return us, w.domain.n_fluid / us, alg


def device_copy(mib: int, reps: int = 20):
    """A plain device-to-device copy (torch copy_): read + write bytes / time."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    dst.copy_(src)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ms = event_time(s, lambda: [dst.copy_(src) for _ in range(reps)])
    del src, dst
    return {"mib": mib, "GBs_read_plus_write": round(2 * n * reps / (ms * 1e-3) / 1e9, 1)}


def adjoint_summary(steps: int = 2000, every: int = 100):
    """The differentiation workload (64x64x48 wetting droplet, FP32 forward,
    `steps` steps): forward time, recorded forward with checkpoints every
    `every` steps plus the reverse sweep of one observable, their ratio, and the
    adjoint gradients of the height h and squared contact radius r2 against
    central finite differences of FP64 runs, at the configured relative step
    1e-4 and at 1e-5."""
    import numpy as np
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd import inputs as I
    w = I.differentiation_case()
    model = w.notes["model"]
    base = dict(abar=w.notes["abar"], kv=w.notes["kv"], eps=w.notes["eps"], tau=w.notes["tau"])
    with iblb.Simulation(w.domain, w.mesh, precision=1, graph=True) as s:
        s.step(64)
        s.sync()
    with iblb.Simulation(w.domain, w.mesh, precision=1, graph=True) as s:
        s.sync()
        t_fwd = event_time(s.stream, lambda: s.step(w.steps)) * 1e-3
    with iblb.Simulation(w.domain, w.mesh, precision=1, graph=True) as s:
        s.sync()
        t0 = time.perf_counter()
        s.adjoint_record(w.steps, every)
        s.sync()
        t_rec = time.perf_counter() - t0
        h, r2, dh, dr2 = iblb.sphere_fit_grad(s.vertices(), 0, w.domain.z_lo, w.mesh.r_cut_wall)
        t0 = time.perf_counter()
        gh, _ = s.adjoint_backward(dh)
        t_bwd = time.perf_counter() - t0
        gr, _ = s.adjoint_backward(dr2)
    ad = {"h": [sum(m * gh[k] for k, m in enumerate(model)), gh[3], gh[4], gh[5]],
          "r2": [sum(m * gr[k] for k, m in enumerate(model)), gr[3], gr[4], gr[5]]}

    def observe(pp):
        wc = I.differentiation_case(pp["abar"], pp["kv"], pp["eps"] / pp["abar"], pp["tau"])
        with iblb.Simulation(wc.domain, wc.mesh, precision=0, graph=True) as sm:
            sm.step(wc.steps)
            hh, rr, _, _ = iblb.sphere_fit_grad(sm.vertices(), 0, wc.domain.z_lo, wc.mesh.r_cut_wall)
        return hh, rr

    names = ("abar", "kv", "eps", "tau")
    errs = {}
    for hrel in (1e-4, 1e-5):
        rel = {"h": [], "r2": []}
        for j, name in enumerate(names):
            hs = base[name] * hrel
            pp, pm = dict(base), dict(base)
            pp[name] += hs
            pm[name] -= hs
            a, b = observe(pp), observe(pm)
            for key, idx in (("h", 0), ("r2", 1)):
                fd = (a[idx] - b[idx]) / (2 * hs)
                rel[key].append(float(abs(ad[key][j] - fd) / max(abs(fd), 1e-300)))
        errs[hrel] = rel
    best = {k: [min(errs[1e-4][k][j], errs[1e-5][k][j]) for j in range(4)] for k in ("h", "r2")}
    return {
        "workload": w.name, "steps": w.steps, "checkpoint_every": every,
        "forward_s": round(t_fwd, 5), "record_s": round(t_rec, 5), "backward_s": round(t_bwd, 5),
        "adjoint_over_forward": round((t_rec + t_bwd) / t_fwd, 3),
        "params": ["abar", "k_V", "eps", "tau"],
        "fd_rel_error_h1e-4": errs[1e-4], "fd_rel_error_h1e-5": errs[1e-5],
        "max_fd_rel_error_h1e-4": max(max(v) for v in errs[1e-4].values()),
        "max_fd_rel_error_best_step": max(max(v) for v in best.values()),
        "h": h, "r2": r2, "grad": {k: [float(x) for x in v] for k, v in ad.items()},
    }


# ----------------------------------------------------------------- CPU oracle

def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(name: str, budget_s: float):
    """Child process: the FP64 oracle on a bounded number of steps of workload
    `name`, at the thread count of OMP_NUM_THREADS; prints one JSON line."""
    from oracle import oracle as O
    w, _ = workload(name)
    sim = O.OracleSim(w.domain, w.mesh)
    sim.step(1)  # warm-up
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        sim.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    print(json.dumps({"mlups": w.domain.n_fluid * steps / dt / 1e6, "steps": steps, "seconds": dt}), flush=True)


def cpu_baseline(name: str, wname: str, budget_s: float):
    """The FP64 oracle on this host's cores and on one core, each in a child
    process that never touches the GPU."""
    nproc = len(os.sched_getaffinity(0))
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or nproc
    legs = {}
    for threads in (cores, 1):
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", name, "--cpu-seconds",
                              str(budget_s)], env=env, capture_output=True, text=True, check=True)
        legs[threads] = json.loads(out.stdout.strip().splitlines()[-1])
    a, one = legs[cores], legs[1]
    return {"value": round(a["mlups"], 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{wname}: {a['steps']} FP64 oracle steps after 1 warm-up step ({a['seconds']:.1f} s) on "
                      f"{cores} threads; {one['steps']} steps ({one['seconds']:.1f} s) on 1 thread",
            "value_1core": round(one["mlups"], 3), "nproc": nproc, "cpu_model": cpu_model()}


def precision_study(steps: int):
    """Equilibrium contact angle of the 128x128x96 wetting droplet with FP32,
    FP16 and BF16 population storage against the FP64 path, at eps/abar =
    0.05, 1 and 7: the same run of `steps` steps in each precision, then the
    sphere fit of the lower contact angle."""
    import torch
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd import inputs as I
    out = {"study": "contact angle vs population storage", "workload": "wetting128", "steps": steps,
           "fit": "sphere fit (method 0) of the vertices >= 2 above the lower wall plane", "cases": []}
    for eps in (0.05, 1.0, 7.0):
        w = I.c3_wetting(eps)
        case = {"eps_over_abar": eps}
        for name in ("fp64", "fp32", "fp16", "bf16"):
            prec = PRECISIONS[name]
            with iblb.Simulation(w.domain, w.mesh, precision=prec, graph=True) as sim:
                sim.step(16)
                sim.sync()
                t0 = time.perf_counter()
                sim.step(steps - 16)
                sim.sync()
                dt = time.perf_counter() - t0
                theta, r, h = sim.contact_angle(0)
                V, _ = sim.volume()
            case[name] = {"theta_deg": theta, "contact_radius": r, "height": h, "volume": V,
                          "mlups": round(w.domain.n_fluid * (steps - 16) / dt / 1e6, 1)}
        for name in ("fp32", "fp16", "bf16"):
            case[name]["dtheta_deg"] = case[name]["theta_deg"] - case["fp64"]["theta_deg"]
        out["cases"].append(case)
        print(json.dumps(case), flush=True)
    print(json.dumps(out), flush=True)


def shear_study(steps: int):
    """Steady deformation D and inclination Theta of a sheared particle at
    Ca = 0.01, 0.05, 0.1, 0.2 on the 64^3 shear domain (walls at -+0.01, R =
    10, level-4 icosphere, Couette start), FP32 storage: the four particles of
    Table 1 with a strain modulus (rigidly and softly coated droplets,
    non-pre-stressed and pure elastic capsules) against the small-deformation
    steady D of Eq. deformation, and a pure droplet abar(1,0,0) against Eq.
    deformation_droplet (35/32 Ca at viscosity ratio 1) and Eq.
    inclination_angle (pi/4 - 35/32 Ca).  D and Theta come from the second
    moments of the polyhedron, sampled 20 times per run; the last 4 samples
    are averaged.  The droplet runs an eighth of the steps and is averaged
    over gammadot t in [0.5, 1]: its relaxation time at viscosity ratio 1 is
    about 2.2 Ca / gammadot, while a mesh with tension
    only (no alpha_2, alpha_3) has no resistance against the tangential drift
    of its vertices that tank-treading accumulates, and its shape creeps
    away from the plateau after about one shear time."""
    import math
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd import inputs as I
    out = {"study": "shear deformation vs small-Ca theory", "workload": "shear64", "steps": steps, "cases": []}
    for kind, shape, nsteps in (("rigidly coated droplet abar(1,1,1)", (1.0, 1.0, 1.0), steps),
                                ("softly coated droplet abar(1,0,1)", (1.0, 0.0, 1.0), steps),
                                ("non-pre-stressed capsule abar(0,1,1)", (0.0, 1.0, 1.0), steps),
                                ("pure elastic capsule abar(0,0,1)", (0.0, 0.0, 1.0), steps),
                                ("droplet abar(1,0,0)", (1.0, 0.0, 0.0), steps // 8)):
        for ca in (0.01, 0.05, 0.1, 0.2):
            w = I.c2_shear(ca)
            abar = w.mesh.alpha[0]
            mesh = I.sphere_mesh(4, 10.0, (31.5, 31.5, 31.5), tuple(abar * k for k in shape))
            gdot = 0.02 / (w.domain.z_hi - w.domain.z_lo)
            case = {"particle": kind, "Ca": ca, "abar": abar, "steps": nsteps, "gammadot_t": gdot * nsteps}
            chunk = nsteps // 20
            trace = []
            try:
                with iblb.Simulation(w.domain, mesh, precision=1, graph=True) as sim:
                    for k in range(20):
                        sim.step(chunk)
                        D, th, _ = sim.shape_dtheta()
                        trace.append((chunk * (k + 1), D, th))
            except iblb.IBLBError as e:
                case["failed_after_step"] = trace[-1][0] if trace else 0
                case["error"] = str(e)
                case["D_trace"] = [round(d, 5) for _, d, _ in trace]
                out["cases"].append(case)
                print(json.dumps(case), flush=True)
                continue
            if shape[2] > 0:
                window = trace[-4:]
            else:
                window = [r for r in trace if 0.5 <= gdot * r[0] <= 1.0]
                case["window_gammadot_t"] = [0.5, 1.0]
            D = sum(d for _, d, _ in window) / len(window)
            th = sum(t for _, _, t in window) / len(window)
            case.update({"D": D, "Theta": th, "D_trace": [round(d, 5) for _, d, _ in trace]})
            if shape[2] > 0:
                # Eq. deformation with the moduli in units of abar and Ca = mu R
                # gammadot / abar (the printed alpha_1 factor cancels, which
                # also covers the non-pre-stressed particles)
                a1, a2, a3 = shape
                k = 5 * (3 * a2 + 4 * a3) / (4 * (3 * a1 * a2 + 5 * a1 * a3 + 2 * a2 * a3 + 2 * a3 * a3))
                case["D_theory"] = k * ca
            else:
                case["D_theory"] = 35.0 / 32.0 * ca
                case["Theta_theory"] = math.pi / 4 - 35.0 / 32.0 * ca
            case["D_rel_err"] = (D - case["D_theory"]) / case["D_theory"]
            out["cases"].append(case)
            print(json.dumps(case), flush=True)
    print(json.dumps(out), flush=True)


def sync_study(rounds: int = 2000):
    """What ordering two whole-GPU phases costs: a kernel boundary (graph-
    replayed launches) against a grid-wide barrier in one cooperative kernel,
    for 256 to 2048 blocks of 256 threads (iblb_probe_phase_sync)."""
    from paper_2305_18919_amd import iblb
    out = {"study": "phase ordering: kernel boundary vs grid-wide barrier", "rounds": rounds, "cases": []}
    for blocks in (256, 512, 1024, 2048):
        try:
            b, g = iblb.probe_phase_sync(blocks, rounds)
            out["cases"].append({"blocks": blocks, "boundary_us": round(b, 3), "barrier_us": round(g, 3)})
        except iblb.IBLBError as e:
            out["cases"].append({"blocks": blocks, "error": str(e)})
        print(json.dumps(out["cases"][-1]), flush=True)
    print(json.dumps(out), flush=True)


def batch_study(steps: int, warmup: int, chunk: int = 500):
    """The 48-domain parameter sweep (cubic edges 32-80, one droplet each)
    stepped as one batch -- each step kernel launched once for all domains,
    launch shape from the library's autotuner -- against the same domains
    stepped one context after another.

    The timed steps run in chunks of `chunk` with a check of every member's
    error word before each chunk: a member that turned unstable is frozen
    there (its garbage state can spread its vertices over the whole domain and
    make every tile active, costing the batch far more than its own share),
    so at most one chunk of its garbage is timed.  MLUPS count the fluid
    nodes of the members stepped in each chunk.  The one-at-a-time leg steps
    the members that stayed stable through the whole batch leg, each replaying
    its own graphs, for the same number of steps.  step_roofline: LB bytes of
    the stable members per step (38 FP32 population accesses per node) over
    the batch's time per step of those members, against 8 TB/s."""
    import torch
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd import inputs as I
    ws = I.batch_sweep()
    sims = [iblb.Simulation(w.domain, w.mesh, precision=1, graph=True) for w in ws]
    out = {"study": "batched sweep", "domains": len(ws), "steps": steps, "warmup": warmup, "check_every": chunk}
    with iblb.Batch(sims) as b:
        t0 = time.perf_counter()
        out["tune_ms_per_step"] = round(b.tune(32), 5)
        out["tune_seconds"] = round(time.perf_counter() - t0, 2)
        out["config"] = b.config
        b.step(warmup)
        status = b.check()
        frozen_before = [k for k, st in enumerate(status) if st != iblb.IBLB_OK]
        dt, node_steps, done, frozen_during = 0.0, 0, 0, []
        while done < steps:
            n = min(chunk, steps - done)
            live = [k for k, st in enumerate(status) if st == iblb.IBLB_OK]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.step(n)
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            node_steps += n * sum(ws[k].domain.n_fluid for k in live)
            done += n
            status = b.check()
            frozen_during += [ws[k].name + f" (by step {warmup + done})" for k in live if status[k] != iblb.IBLB_OK]
    stable = [k for k, st in enumerate(status) if st == iblb.IBLB_OK]
    nodes = sum(ws[k].domain.n_fluid for k in stable)
    mlups = node_steps / dt / 1e6
    ms = nodes / (mlups * 1e6) * 1e3  # batch time per step of the stable members
    out.update({
        "frozen_before_timing": [ws[k].name for k in frozen_before],
        "frozen_during_timing": frozen_during,
        "stable_members": len(stable), "fluid_nodes": nodes, "vertices": sum(ws[k].mesh.n_vertices for k in stable),
        "batch": {"ms_per_step": round(ms, 5), "mlups": round(mlups, 1)},
    })
    alg = nodes * lb_bytes_per_node(1)
    out["step_roofline"] = {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "alg_bytes_per_step": alg}
    seq = 0.0
    for k in stable:
        s = sims[k]
        s.step(32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t0
    seq_mlups = nodes * steps / seq / 1e6
    out["one_at_a_time"] = {"ms_per_step": round(seq * 1e3 / steps, 5), "mlups": round(seq_mlups, 1)}
    out["speedup"] = round(mlups / seq_mlups, 2)
    for s in sims:
        s.close()
    print(json.dumps(out), flush=True)


def wetting_study(steps: int):
    """Equilibrium contact angle against eps/abar for the five models of
    Table 1: the pre-stressed pure, softly and rigidly coated droplets at
    eps/abar in {0.05, 1, 3, 5, 7}, and the non-pre-stressed pure elastic and
    non-pre-stressed capsules at eps/abar in {0.05, 0.5, 1, 1.5, 2} (they
    stay stable over a narrower range); 64x64x48, R = 12 at level 4, abar =
    1e-3 (inertial-capillary time sqrt(R^3/abar) = 1314 steps), all 25 runs
    in one batch.
    theta from the sphere fit is sampled 10 times; the paper's fit of Eq.
    cos_theta_prediction with its Table 1 constants (other R and mesh) is
    listed beside it."""
    import math
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd import inputs as I
    pre, non = (0.05, 1.0, 3.0, 5.0, 7.0), (0.05, 0.5, 1.0, 1.5, 2.0)
    fits = {"pure droplet": ((1.0, 0.0, 0.0), (0.78, 0.42, 0.0, 1.0), pre),
            "softly coated": ((1.0, 0.0, 1.0), (0.87, 0.5, 0.0, 1.0), pre),
            "rigidly coated": ((1.0, 1.0, 1.0), (0.91, 0.55, 0.0, 1.0), pre),
            "pure elastic capsule": ((0.0, 0.0, 1.0), (0.71, 2.0, 0.2, 0.75), non),
            "non-pre-stressed capsule": ((0.0, 1.0, 1.0), (0.7, 1.6, 0.2, 0.75), non)}
    cases, sims = [], []
    for name, (model, _, ratios) in fits.items():
        for r in ratios:
            w = I.wetting_case(model, r)
            cases.append((name, r))
            sims.append(iblb.Simulation(w.domain, w.mesh, precision=1, graph=True))
    trace = [[] for _ in cases]
    with iblb.Batch(sims) as b:
        b.tune(32)
        chunk = max(16, steps // 10 // 16 * 16)
        for _ in range(10):
            b.step(chunk)
            status = b.check()
            for k, s in enumerate(sims):
                if status[k] == iblb.IBLB_OK:
                    th, rr, hh = s.contact_angle(0)
                    trace[k].append(round(th, 2))
    out = {"study": "equilibrium contact angle vs eps/abar", "steps": 10 * chunk, "R": 12.0, "abar": 1e-3,
           "cases": []}
    for k, (name, r) in enumerate(cases):
        a, bb, c, d = fits[name][1]
        cos_fit = max(-1.0, min(1.0, a * math.atan(bb * (r - c)) - d))
        out["cases"].append({"model": name, "eps_over_abar": r, "status": status[k],
                             "theta_deg": trace[k][-1] if trace[k] else None, "theta_trace": trace[k],
                             "paper_fit_theta_deg": round(math.degrees(math.acos(cos_fit)), 1)})
    for s in sims:
        s.close()
    print(json.dumps(out), flush=True)


def precision64_study(steps: int):
    """Equilibrium contact angle per population storage near equilibrium: the
    softly coated droplet abar(1,0,1) of the 64x64x48 wetting case (R = 12,
    abar = 1e-3) at eps/abar = 0.05, 1 and 7, `steps` steps in FP64, FP32,
    FP16 and BF16 storage (one batch of the three runs per storage), then the
    sphere fit of the lower contact angle and its difference from FP64."""
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd import inputs as I
    ratios = (0.05, 1.0, 7.0)
    out = {"study": "contact angle vs population storage", "workload": "wetting64x48", "steps": steps,
           "model": "softly coated abar(1,0,1)", "abar": 1e-3, "R": 12.0,
           "fit": "sphere fit (method 0) of the vertices >= 2 above the lower wall plane", "cases": []}
    res = {}
    ws = [I.wetting_case((1.0, 0.0, 1.0), r) for r in ratios]
    for name in ("fp64", "fp32", "fp16", "bf16"):
        sims = [iblb.Simulation(w.domain, w.mesh, precision=PRECISIONS[name], graph=True) for w in ws]
        with iblb.Batch(sims) as b:
            b.step(steps)
            status = b.check()
        for k, r in enumerate(ratios):
            if status[k] == iblb.IBLB_OK:
                th, cr, h = sims[k].contact_angle(0)
                V, _ = sims[k].volume()
                res[(name, r)] = {"theta_deg": th, "contact_radius": cr, "height": h, "volume": V}
            else:
                res[(name, r)] = {"status": int(status[k])}
        for s in sims:
            s.close()
    for r in ratios:
        case = {"eps_over_abar": r}
        for name in ("fp64", "fp32", "fp16", "bf16"):
            case[name] = res[(name, r)]
            if name != "fp64" and "theta_deg" in case[name] and "theta_deg" in case["fp64"]:
                case[name]["dtheta_deg"] = case[name]["theta_deg"] - case["fp64"]["theta_deg"]
                case[name]["dheight"] = case[name]["height"] - case["fp64"]["height"]
        out["cases"].append(case)
    print(json.dumps(out), flush=True)


def spreading_study(steps: int):
    """Spreading of a pure droplet abar(1,0,0) on the wetting wall (Eq.
    tanner_law): the 64x64x48 wetting case (R = 12, abar = 1e-3, t* =
    sqrt(R^3/abar) = 1314 steps) at eps/abar = 1, 3, 5 and 7 in one FP32
    batch.  The contact radius r (the equivalent radius of the faces within
    one lattice unit of the wall plane) is sampled at log-spaced times up to
    `steps`; delta and C of r/R = C (t/t*)^delta are fitted over t/t* >= 0.2
    up to the time r first reaches 90 % of its largest value."""
    import math
    import numpy as np
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd import inputs as I
    from paper_2305_18919_amd.analysis import contact_patch_radius, power_law_fit
    ratios = (1.0, 3.0, 5.0, 7.0)
    abar, R = 1e-3, 12.0
    t_star = math.sqrt(R ** 3 / abar)
    ws = [I.wetting_case((1.0, 0.0, 0.0), r, abar=abar) for r in ratios]
    sims = [iblb.Simulation(w.domain, w.mesh, precision=1, graph=True) for w in ws]
    times = sorted({int(round(x / 16.0)) * 16 for x in np.geomspace(16, steps, 48)} - {0})
    z_wall = ws[0].domain.z_lo
    r_t = [[] for _ in ratios]
    with iblb.Batch(sims) as b:
        t = 0
        for tn in times:
            b.step(tn - t)
            t = tn
            status = b.check()
            for k, s in enumerate(sims):
                r_t[k].append(contact_patch_radius(s.vertices(), ws[k].mesh.faces, z_wall)
                              if status[k] == iblb.IBLB_OK else float("nan"))
        theta = [s.contact_angle(0)[0] if status[k] == iblb.IBLB_OK else None for k, s in enumerate(sims)]
    out = {"study": "spreading law", "workload": "wetting64x48", "model": "pure droplet abar(1,0,0)",
           "R": R, "abar": abar, "t_star": t_star, "steps": times[-1], "t": times, "cases": []}
    for k, r in enumerate(ratios):
        rr = np.array(r_t[k])
        case = {"eps_over_abar": r, "status": int(status[k]), "theta_final_deg": theta[k],
                "r_over_R": [round(v / R, 5) for v in rr]}
        if status[k] == iblb.IBLB_OK:
            case.update(power_law_fit(np.array(times, dtype=float), rr, R, t_star))
        out["cases"].append(case)
    for s in sims:
        s.close()
    print(json.dumps(out), flush=True)


def adjoint_study(every: int):
    """The differentiation workload (64x64x48, pure droplet R = 12, level 4,
    abar = 1e-3, eps/abar = 1, 2000 steps, FP32 populations): gradients of
    the final height h and signed squared contact radius r2 of the fit with
    respect to (abar, k_V, eps, tau) by the hand-written adjoint, timed against
    the forward run alone, and checked against central differences of the
    FP64 path (relative steps 1e-4 for abar and k_V, 1e-5 for eps and tau: the
    plainly cut-off wall force makes the observables only piecewise smooth,
    and wider steps in the parameters the contact region is most sensitive to
    straddle its switching)."""
    import numpy as np
    import torch
    from paper_2305_18919_amd import iblb
    from paper_2305_18919_amd import inputs as I
    w = I.differentiation_case()
    model = w.notes["model"]
    base = dict(abar=w.notes["abar"], kv=w.notes["kv"], eps=w.notes["eps"], tau=w.notes["tau"])
    out = {"study": "adjoint", "workload": w.name, "steps": w.steps,
           "fluid_nodes": w.domain.n_fluid, "vertices": w.mesh.n_vertices}
    # forward alone (graph-replayed steps)
    with iblb.Simulation(w.domain, w.mesh, precision=1, graph=True) as s:
        s.step(64)  # warm-up: code objects loaded, graph path exercised
        torch.cuda.synchronize()
    with iblb.Simulation(w.domain, w.mesh, precision=1, graph=True) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(w.steps)
        s.sync()
        t_fwd = time.perf_counter() - t0
    # recorded forward, then the reverse sweep (one per observable): every
    # time level kept (every = 0), and checkpoints every `every` steps with
    # recompute
    modes, grads = {}, {}
    for ev in (0, every):
        with iblb.Simulation(w.domain, w.mesh, precision=1, graph=True) as s:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.adjoint_record(w.steps, ev)
            s.sync()
            t_rec = time.perf_counter() - t0
            h, r2, dh, dr2 = iblb.sphere_fit_grad(s.vertices(), 0, w.domain.z_lo, w.mesh.r_cut_wall)
            t0 = time.perf_counter()
            gh, _ = s.adjoint_backward(dh)
            t_bwd = time.perf_counter() - t0
            gr, _ = s.adjoint_backward(dr2)
        modes[ev] = {"record_s": round(t_rec, 4), "backward_s": round(t_bwd, 4),
                     "adjoint_over_forward": round((t_rec + t_bwd) / t_fwd, 3)}
        grads[ev] = (gh, gr)
    t_rec, t_bwd = modes[0]["record_s"], modes[0]["backward_s"]
    gh, gr = grads[0]
    ad = {"h": [sum(m * gh[k] for k, m in enumerate(model)), gh[3], gh[4], gh[5]],
          "r2": [sum(m * gr[k] for k, m in enumerate(model)), gr[3], gr[4], gr[5]]}

    def observe(pp):
        wc = I.differentiation_case(pp["abar"], pp["kv"], pp["eps"] / pp["abar"], pp["tau"])
        with iblb.Simulation(wc.domain, wc.mesh, precision=0, graph=True) as sm:
            sm.step(wc.steps)
            hh, rr, _, _ = iblb.sphere_fit_grad(sm.vertices(), 0, wc.domain.z_lo, wc.mesh.r_cut_wall)
        return hh, rr

    fd = {"h": [], "r2": []}
    for name in ("abar", "kv", "eps", "tau"):
        hstep = base[name] * (1e-5 if name in ("eps", "tau") else 1e-4)
        pp, pm = dict(base), dict(base)
        pp[name] += hstep
        pm[name] -= hstep
        a, b = observe(pp), observe(pm)
        fd["h"].append((a[0] - b[0]) / (2 * hstep))
        fd["r2"].append((a[1] - b[1]) / (2 * hstep))
    rel = {k: [abs(ad[k][j] - fd[k][j]) / abs(fd[k][j]) for j in range(4)] for k in ad}
    out.update({
        "h": h, "r2": r2, "params": ["abar", "k_V", "eps", "tau"],
        "adjoint": ad, "finite_difference_fp64": fd, "rel_error": rel,
        "max_rel_error": max(max(v) for v in rel.values()),
        "forward_s": round(t_fwd, 4), "record_s": t_rec, "backward_s": t_bwd,
        "adjoint_over_forward": round((t_rec + t_bwd) / t_fwd, 3),
        "backward_over_forward": round(t_bwd / t_fwd, 3),
        "storage": "every time level in device memory (FP32 populations, 19 x nodes x 4 B per level)",
        "checkpoint_mode": dict(modes[every], checkpoint_every=every,
                                max_rel_diff_from_every_level_kept=max(
                                    float(np.max(np.abs(np.array(grads[every][j]) - np.array(grads[0][j])) /
                                                 np.maximum(np.abs(np.array(grads[0][j])), 1e-300)))
                                    for j in (0, 1))),
    })
    print(json.dumps(out), flush=True)


def copy_pass(mib: int, reps: int):
    """A plain device-to-device copy of `mib` MiB, `reps` times (counter calibration)."""
    import torch
    n = mib * (1 << 20)
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pass": "copy", "bytes_read_per_copy": n, "bytes_written_per_copy": n, "copies": reps}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="wetting128")
    ap.add_argument("--timed-steps", type=int, default=200, help="steps of the per-dispatch hipEvent pass")
    ap.add_argument("--lb-launches", type=int, default=800, help="launches of the LB-only pass")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the timed step and its roofline (no secondary figures, adjoint or oracle)")
    ap.add_argument("--cpu-leg", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--pass", dest="only", choices=["lb", "copy", "step"], default=None)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--study", choices=["precision", "precision64", "shear", "batch", "adjoint", "wetting",
                                        "spreading", "sync"], default=None,
                    help="precision: contact angle of the 128x128x96 wetting droplet per population storage; "
                         "precision64: the same on the 64x64x48 wetting case, near equilibrium; "
                         "shear: steady D and Theta against the small-Ca theory; "
                         "wetting: equilibrium contact angle against eps/abar for the five models; "
                         "spreading: contact radius against time (Eq. tanner_law); "
                         "sync: kernel boundary against grid-wide barrier")
    ap.add_argument("--study-steps", type=int, default=50000)
    ap.add_argument("--precision", choices=sorted(PRECISIONS), default=None,
                    help="population storage (default: the workload's, FP32 for the benchmark workloads)")
    args = ap.parse_args()
    if args.cpu_leg is not None:
        cpu_leg(args.cpu_leg, args.cpu_seconds)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the library has no multi-GPU path "
                                   "(the sharding design is described with the kernels)"}))
        raise SystemExit(2)

    import torch
    from paper_2305_18919_amd import iblb

    studies = {"precision": lambda: precision_study(args.study_steps),
               "shear": lambda: shear_study(args.study_steps),
               "batch": lambda: batch_study(args.study_steps, args.warmup),
               "adjoint": lambda: adjoint_study(100),
               "wetting": lambda: wetting_study(args.study_steps),
               "precision64": lambda: precision64_study(args.study_steps),
               "spreading": lambda: spreading_study(args.study_steps),
               "sync": lambda: sync_study()}
    if args.study is not None:
        studies[args.study]()
        return
    w, prec = workload(args.workload)
    if args.precision is not None:
        prec = PRECISIONS[args.precision]
        if prec != 1:
            w.name = w.name.replace("_f32", "") + f"_{args.precision}"
    dom, mesh = w.domain, w.mesh
    if args.only == "copy":
        copy_pass(args.copy_mib, 10)
        return
    if args.only == "lb":
        print(json.dumps({"pass": "lb", "workload": w.name, "lb_only": lb_roofline(dom, prec, args.lb_launches)}),
              flush=True)
        return

    # the timed step: graphs captured at construction, W warm-up steps, then
    # exactly K steps between hipEvents on the library stream
    sim = iblb.Simulation(dom, mesh, precision=prec, graph=True)
    split = sim.lb_split()
    sim.step(args.warmup)
    sim.sync()
    q0 = sim.vertices()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = event_time(sim.stream, lambda: sim.step(args.steps))
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ms / args.steps
    mlups = dom.n_fluid * args.steps / (ms * 1e-3) / 1e6
    print(f"[bench] {w.name}: {ms_per_step * 1e3:.2f} us/step, {mlups:.1f} MLUPS", file=sys.stderr, flush=True)

    geo = step_geometry(dom, q0, split)
    alg = algorithmic_bytes(dom, mesh, prec, geo)
    achieved = alg["total"] / (ms_per_step * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": step_traffic(w.name, prec),
                "kernel": "whole step (forces, spread, moments, move dispatches)",
                "alg_bytes_per_step": alg["total"], "alg_bytes_lb": alg["lb"], "alg_bytes_ib": alg["ib"],
                "avg_us": round(ms_per_step * 1e3, 3)}

    # per-dispatch pass: the same four dispatches launched one by one, each
    # bracketed by hipEvents
    dispatches = {}
    if args.only != "step":
        sim.set_timing(True)
        sim.reset_timing()
        sim.step(args.timed_steps)
        sim.sync()
        for name in DISPATCHES:
            tms, n = sim.kernel_time(name)
            if n:
                us = tms * 1e3 / n
                b = alg["per_dispatch"][name]
                dispatches[name] = {"avg_us": round(us, 3), "launches": n, "alg_bytes": b,
                                    "lb_nodes": geo["lb_nodes"][name],
                                    "achieved_GBs": round(b / (us * 1e-6) / 1e9, 1)}
        sim.set_timing(False)
        if dispatches:
            dom_name = max(dispatches, key=lambda k: dispatches[k]["avg_us"])
            roofline["dominant_dispatch"] = dom_name
    active_nodes = sim.active_nodes()
    sim.close()

    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": w.name, "grid": [dom.nx, dom.ny, dom.nz], "fluid_nodes": dom.n_fluid,
                   "vertices": mesh.n_vertices, "faces": mesh.n_faces, "tau": dom.tau,
                   "alpha": list(mesh.alpha), "positions": "f64",
                   "launch": "hipGraphs of 16 and 1 steps captured before the warm-up", "lb_split": split},
        "roofline": roofline,
        "wall_ms_per_step": round(wall * 1e3 / args.steps, 6),
        "dispatches": dispatches,
        "geometry": dict({k: v for k, v in geo.items() if k != "lb_nodes"}, active_tile_nodes_device=active_nodes,
                         lb_nodes=geo["lb_nodes"]),
    }
    if not args.no_extra and args.only != "step":
        out["lb_only"] = lb_roofline(dom, prec, args.lb_launches)
        pw = probe256()
        out["probe256"] = {"lb_only": lb_roofline(pw.domain, 1, 64)}
        us, ml, alg = coupled_rate(pw, 1, 64, 16)
        # beyond the Infinity Cache: the whole step against the HBM peak
        out["probe256"]["coupled_step"] = {"avg_us": round(us, 3), "mlups": round(ml, 1), "alg_bytes_per_step": alg,
                                           "achieved_GBs": round(alg / (us * 1e-6) / 1e9, 1),
                                           "frac": round(alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
        out["device_copy"] = [device_copy(128), device_copy(1024)]
        out["adjoint"] = adjoint_summary()
    if not args.no_cpu and args.only != "step":
        out["cpu_baseline"] = cpu_baseline(args.workload, w.name, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
