"""Benchmark of the fused finite-volume TVD-RK3 stage on one MI355X.

Workload (default): compressible Navier-Stokes Taylor-Green vortex, Ma 0.1,
Re 1600, Pr 0.72, constant viscosity, periodic 256^3, FP64, seeded +-1e-3
velocity noise, WENO5-Z + HLLC + 4th-order viscous fluxes, TVD-RK3 at CFL 0.5.
One timed "step" = the three fused stage kernels, the third also reducing
the CFL time step of its output for the next step (the whole hot path).  Inputs are generated on the device and
resident in HBM before timing starts.

Prints one JSON line.  ``value`` is cell-updates per second counted per RK
stage (cells x 3 x steps / time).  ``roofline`` reports the stage kernel:
its algorithmic FP64 operations per cell (counted from the scheme's formulas,
see FLOPS_PER_CELL) times cells, over its mean duration measured with HIP
events on the launch stream, against the MI355X FP64 vector peak; the HBM
view (algorithmic bytes over the same duration) is reported beside it.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import struct
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector
# MI355X FP32 vector: 157.3 TFLOP/s is the packed (two-wide) rate; the library is built
# without packed FP32 operations, so its FP32 kernels issue at the FP64 vector rate
PEAK_FP32_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
# VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second
PEAK_VALU_LANE_INSTS = 256 * 4 * 16 * 2.4e9

# Algorithmic floating-point operations per cell per stage (+ - * / sqrt min
# max abs and comparisons each count 1), from the formulas of the scheme:
#   WENO5-Z pair (both face values of a cell, one component, one direction): 95
#   one-sided WENO5-Z value: 72;  TENO6-A face (both states, shared cut-off): 389
#   characteristic projection of a face: 30 + 12 per projected field + 6 per component
#   HLLC face: 91;  viscous face: 80 (sixth order: 120);  cell-centred derivatives: 9 x 5;
#   U -> W: 13 (+1 for T = p/rho);  divergence: 9 per component;  Shu-Osher combine: 5 per component.
def flops_per_cell(model: int, recon: int = 0, scheme: int = 0, visc_order: int = 4) -> int:
    nc = 7 if model == 2 else 5
    if scheme == 1:
        per_face = 389 * nc
    elif recon == 1:
        per_face = 2 * 72 * nc
    else:
        per_face = 95 * nc
    if recon == 1:
        per_face += 30 + 12 * (2 + (2 if model == 2 else 1)) + 6 * nc
    weno = per_face * 3
    hllc = 91 * 3 + (2 * 3 * 3 if model == 2 else 0)
    visc = (80 * 3 + 45) if model == 1 else 0
    if model == 1 and visc_order == 6:
        # separate passes: q (13), gradient (9 x 9), two faces per direction (2 x 3 x 120) + divergence (12)
        visc = 13 + 81 + 720 + 12
    conv = 13 + (1 if model == 1 else 0) + (10 if model == 2 else 0)
    div = 9 * nc + (7 if model == 2 else 0)
    rk = 5 * nc
    return weno + hllc + visc + conv + div + rk


PROFILES_DIR = os.path.join(ROOT, "profiles")


# the benchmarked instantiation: stage_kernel<double, NS, positivity off, primitive
# reconstruction, constant viscosity, 16x16 tile, 256 threads>
STAGE_KERNEL_SYMBOL = "_ZN2fv12stage_kernelIdLi1ELi0ELi0ELi0ELi16ELi16ELi256EEEvNS_9StageArgsIT_EE"
# the stage instantiation each workload with committed counter records runs: the NS
# default above, and the five-equation shock-bubble's <double, DIM, limiters on,
# primitive reconstruction, no THINC, 16x16 tile, 256 threads>
WORKLOAD_KERNELS = {
    "ns-f64-256": STAGE_KERNEL_SYMBOL,
    "dim-f64-256": "_ZN2fv12stage_kernelIdLi2ELi1ELi0ELi0ELi16ELi16ELi256EEEvNS_9StageArgsIT_EE",
}


def _elf_sections(elf: bytes):
    shoff, = struct.unpack_from("<Q", elf, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", elf, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", elf, shoff + i * shentsize) for i in range(shnum)]
    names = secs[shstrndx][4]
    return [(elf[names + s[0]:elf.index(b"\0", names + s[0])].decode(), s) for s in secs]


def stage_kernel_hash(symbol: str = STAGE_KERNEL_SYMBOL) -> str:
    """Fingerprint of the benchmarked stage kernel (or of another kernel of the library,
    by its mangled name): a hash of its gfx950 machine code and kernel descriptor
    (register and LDS allocation), read from the code objects bundled in the built
    library.  Unrelated changes to the sources (other template instantiations) leave it
    unchanged; any change to this kernel changes it."""
    from paper_2402_05193_amd import solver as S
    with open(S.LIB_PATH, "rb") as fh:
        so = fh.read()
    fat = next(so[s[4]:s[4] + s[5]] for nm, s in _elf_sections(so) if nm == ".hip_fatbin")
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    h = hashlib.sha256()
    found = 0
    pos = fat.find(magic)
    while pos >= 0:
        n, = struct.unpack_from("<Q", fat, pos + len(magic))
        p = pos + len(magic) + 8
        for _ in range(n):
            off, size, tl = struct.unpack_from("<QQQ", fat, p)
            triple = fat[p + 24:p + 24 + tl].decode()
            p += 24 + tl
            if "gfx950" not in triple:
                continue
            co = fat[pos + off:pos + off + size]
            secs = _elf_sections(co)
            for _, sym in secs:
                if sym[1] != 2:      # SHT_SYMTAB
                    continue
                strtab = secs[sym[6]][1][4]
                for k in range(sym[5] // 24):
                    name_off, info, _, shndx, value, ssize = struct.unpack_from("<IBBHQQ", co, sym[4] + k * 24)
                    name = co[strtab + name_off:co.index(b"\0", strtab + name_off)].decode()
                    if name in (symbol, symbol + ".kd"):
                        sec = secs[shndx][1]
                        start = sec[4] + value - sec[3]
                        body = bytearray(co[start:start + ssize])
                        if name.endswith(".kd"):
                            body[16:24] = bytes(8)   # code entry offset: depends on the layout only
                        h.update(bytes(body))
                        found += 1
        pos = fat.find(magic, pos + len(magic))
    if found != 2:
        raise RuntimeError(f"kernel {symbol} not found in the built library")
    return h.hexdigest()[:16]


def _profile_record(kind: str, workload_key: str):
    """The numbers of a record line ('<kind>-record: kernel=<fingerprint> workload=<key>
    name=value ...') of a committed rocprofv3 summary under profiles/, if it was taken on
    the workload's current stage kernel (same fingerprint); else None."""
    symbol = WORKLOAD_KERNELS.get(workload_key)
    if symbol is None or not os.path.isdir(PROFILES_DIR):
        return None
    want = stage_kernel_hash(symbol)
    pat = re.compile(kind + r"-record: kernel=(\w+) workload=(\S+)((?: \w+=[\d.e+-]+)+)")
    for path in sorted(glob.glob(os.path.join(PROFILES_DIR, "*.md"))):
        with open(path) as fh:
            for line in fh:
                m = pat.search(line)
                if m and m.group(1) == want and m.group(2) == workload_key:
                    return {k: float(v) for k, v in re.findall(r"(\w+)=([\d.e+-]+)", m.group(3))}
    return None


def measured_traffic(workload_key: str):
    """HBM bytes per stage-kernel launch (FETCH_SIZE + WRITE_SIZE, scaled by a copy
    kernel of known size) recorded in the committed rocprofv3 summary for the current
    kernel and workload; else None."""
    r = _profile_record("traffic", workload_key)
    return int(r["fetch_bytes"] + r["write_bytes"]) if r else None


def measured_valu_insts_per_cell(workload_key: str):
    """VALU lane-instructions per cell and launch (SQ_INSTS_VALU x 64 / cells) recorded in
    the committed rocprofv3 summary for the current kernel and workload; else None."""
    r = _profile_record("valu", workload_key)
    return r["insts_per_cell"] if r else None


def bytes_per_cell(nc: int, es: int, stage: int) -> int:
    # stage 1 reads U^n and writes U^(1); stages 2-3 read U^n, U^(k) and write one array
    return (2 if stage == 1 else 3) * nc * es


def _native_oracle():
    """The oracle's source built for this host (-O3 -march=native, contraction off, so
    the same results as the reference build), into a temporary directory; None if the
    host has no C compiler."""
    import subprocess
    import tempfile
    import oracle as O
    out = os.path.join(tempfile.mkdtemp(prefix="oracle_native_"), "liboracle_native.so")
    try:
        subprocess.run(["make", "-s", "-C", os.path.join(ROOT, "oracle"), "-B", "native", f"NATIVE_OUT={out}"],
                       check=True, capture_output=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    O._lib = O._load(out)
    return out


def run_oracle_baseline(n: int, model: int) -> dict:
    """The FP64 oracle timed on this host's cores on bounded samples of the workload:
    one full TVD-RK3 step (three right-hand sides) of the benchmarked problem, plus one
    step of its smaller sizes (C1 32^3 Euler, 128^3, and the 256 x 128 x 128
    five-equation shock-bubble), and a 64^3 step on one thread."""
    import oracle as O
    from paper_2402_05193_amd import workloads as WL
    native = _native_oracle()
    threads = O.max_threads()

    def one_step(case):
        cfg = O.Config(**case.cfg_kwargs())
        U = O.prim_to_cons(cfg, case.W)
        dt = O.compute_dt(cfg, U, 0.5)
        t0 = time.perf_counter()
        O.rk3_step(cfg, U, dt)
        return cfg.nx * cfg.ny * cfg.nz * 3 / (time.perf_counter() - t0), time.perf_counter() - t0

    if model == 2:
        main_case = WL.shock_bubble(256, 128, 128) if n >= 256 else WL.shock_bubble(2 * n, n // 2, n // 2)
    else:
        main_case = WL.taylor_green(n, viscous=(model == 1))
    value, el = one_step(main_case)
    samples = {}
    for name, case in (("c1_euler_tgv32", WL.taylor_green(32)),
                       ("ns_tgv128", WL.taylor_green(128, viscous=True)),
                       ("dim_sbi256x128x128", WL.shock_bubble(256, 128, 128))):
        if name.startswith("dim") and model == 2 and n >= 256:
            continue
        v, t = one_step(case)
        samples[name] = {"value": v, "seconds": t}
    # one thread, a 64^3 block of the workload's kind
    small = WL.taylor_green(64, viscous=(model == 1)) if model != 2 else WL.shock_bubble(64, 32, 32)
    O.set_threads(1)
    try:
        v1, el1 = one_step(small)
    finally:
        O.set_threads(threads)
    model_name = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model_name = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": value, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"one TVD-RK3 step (3 stages) of the same workload, {main_case.nx}x{main_case.ny}x{main_case.nz} "
                      f"FP64, {el:.1f} s on {threads} threads",
            "build": "-O3 -march=native -ffp-contract=off (built on this host)" if native
                     else "-O3 -ffp-contract=off (no compiler on this host for a native build)",
            "other_samples": samples,
            "single_thread": {"value": v1, "sample": f"one TVD-RK3 step at {small.nx}x{small.ny}x{small.nz}, "
                                                     f"{el1:.1f} s on 1 thread"},
            "cpu_model": model_name}


def run_serving(n_req: int, rate: float, max_batch: int, pool_gib: float, seed: int = 2402,
                low_rate: float = 20.0, low_n: int = 80, fill: int | None = 768, use_graph: bool = True,
                policy: str = "srpt", backlog: int | None = 8, protect_oldest: bool = False) -> dict:
    """Serving benchmark: a seeded Poisson stream of independent 3-D Riemann problems
    (single- and two-phase, grids 64^3 .. 256x128x128, 50 RK3 steps each, FP32, CFL 0.5),
    served by continuous batching (graph replay; admission by memory and, with fill, by
    GPU fill: a request joins the running batch while the batch's stage workgroups are
    below the budget) and one request at a time; at the offered rate of the workload
    (above what one GPU sustains, so latencies are queueing-dominated) and at a lower
    rate both paths can sustain."""
    from paper_2402_05193_amd import serving as SV
    from paper_2402_05193_amd import workloads as WL

    srv = SV.Server(pool_bytes=int(pool_gib * (1 << 30)), max_batch=max_batch, use_graph=use_graph,
                    fill_workgroups=fill, policy=policy, backlog=backlog, protect_oldest=protect_oldest)
    # warm-up: every kernel variant once on both paths (tiny grids)
    warm = lambda: [SV.job_from_request(WL.riemann_request(i, seed + 1, grids=((16, 16, 16),), steps=2), 0.0)
                    for i in range(6)]
    srv.run_batched(warm())
    srv.run_sequential(warm())

    def stream(r, n):
        arrivals = WL.poisson_arrivals(n, r, seed)
        reqs = [WL.riemann_request(i, seed) for i in range(n)]
        res = {"arrival_rate_per_s": r, "requests": n}
        for mode in ("batched", "sequential"):
            jobs = [SV.job_from_request(q, a) for q, a in zip(reqs, arrivals)]
            st = srv.run_batched(jobs) if mode == "batched" else srv.run_sequential(jobs)
            res[mode] = st.summary()
            print(f"[bench] serving {r:g}/s {mode}: {json.dumps(res[mode])}", flush=True)
        res["throughput_ratio_batched_vs_sequential"] = (res["batched"]["cell_updates_per_s"] /
                                                         res["sequential"]["cell_updates_per_s"])
        return res

    main = stream(rate, n_req)
    low = stream(low_rate, low_n) if low_n > 0 else None
    srv.close()
    out = {"workload": f"Poisson stream of planar 3-D Riemann problems (Euler / five-equation air-helium, "
                       f"grids {list(WL.SERVING_GRIDS)}), 50 TVD-RK3 steps each at CFL 0.5, FP32, limiters on",
           "max_batch": max_batch, "pool_gib": pool_gib, "fill_workgroups": fill, "policy": policy,
           "backlog": backlog, "protect_oldest": protect_oldest,
           "offered": main,
           "graphs_cached": srv.batch.graph_count()}
    if low is not None:
        out["sustainable"] = low
    out["p50_latency_s"] = main["batched"]["p50_latency_s"]
    out["p99_latency_s"] = main["batched"]["p99_latency_s"]
    out["throughput_ratio_batched_vs_sequential"] = main["throughput_ratio_batched_vs_sequential"]
    return out


def run_adjoint_bench(n: int = 64, nsteps: int = 100, every: int = 10) -> dict:
    """Differentiation workload: gradient of the kinetic energy after nsteps fixed-dt
    TVD-RK3 steps of 64^3 decaying turbulence (Euler, FP64, WENO-Z eps 1e-6) with
    respect to the initial state, through the hand-written adjoint with checkpoints."""
    import math
    import torch
    from paper_2402_05193_amd import adjoint as AD
    from paper_2402_05193_amd import solver as S
    from paper_2402_05193_amd import workloads as WL

    h = 2 * math.pi / n
    cfg = S.Config(nx=n, ny=n, nz=n, dx=h, dy=h, dz=h, model=S.EULER, dtype=S.F64, weno_eps=1e-6, cfl=0.5)
    W = torch.from_numpy(WL.decaying_turbulence(n, seed=0)).cuda()
    U = S.empty_state(cfg)
    S.prim_to_cons(cfg, W, U)
    ws = S.workspace(cfg)
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    S.compute_dt(cfg, U, dtd, ws)
    dt = float(dtd)
    Rbar = torch.randn(U.shape, dtype=torch.float64, device="cuda")
    Ubar = torch.empty_like(U)
    for _ in range(3):
        S.rhs_adjoint(cfg, U, Rbar, Ubar)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        S.rhs_adjoint(cfg, U, Rbar, Ubar)
    e1.record()
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1) / reps
    R = torch.empty_like(U)
    e0.record()
    for _ in range(reps):
        S.rhs(cfg, U, R)
    e1.record()
    torch.cuda.synchronize()
    rhs_ms = e0.elapsed_time(e1) / reps
    # forward alone, then forward + backward of the whole trajectory
    fwd = []
    for r in range(4):
        X = U.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.advance(cfg, X, nsteps, dt, ws)
        torch.cuda.synchronize()
        if r > 0:
            fwd.append(time.perf_counter() - t0)
    fwd_s = sorted(fwd)[1]
    # forward + gradient: one untimed run (kernels loaded, workspaces allocated), then the
    # median of three timed runs
    runs = []
    for r in range(4):
        U0 = U.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = AD.kinetic_energy(cfg, AD.advance_fixed_dt(cfg, U0, nsteps, dt, every=every))
        (g,) = torch.autograd.grad(L, U0)
        torch.cuda.synchronize()
        if r > 0:
            runs.append(time.perf_counter() - t0)
    grad_s = sorted(runs)[1]
    return {"workload": f"gradient of kinetic energy after {nsteps} fixed-dt TVD-RK3 steps, {n}^3 decaying "
                        f"turbulence (Euler, FP64, WENO-Z eps 1e-6), checkpoints every {every} steps",
            "rhs_adjoint_ms": adj_ms, "rhs_ms": rhs_ms, "adjoint_over_rhs": adj_ms / rhs_ms,
            "forward_s": fwd_s, "forward_plus_gradient_s": grad_s, "gradient_over_forward": grad_s / fwd_s,
            "timing": "median of 3 runs after one untimed run",
            "loss": float(L), "grad_finite": bool(torch.isfinite(g).all().item())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--model", choices=["ns", "euler", "dim"], default="ns")
    ap.add_argument("--recon", type=int, choices=[0, 1], default=0,
                    help="reconstruction variables: 0 primitive (the benchmark), 1 characteristic")
    ap.add_argument("--scheme", type=int, choices=[0, 1], default=0,
                    help="reconstruction scheme: 0 WENO5-Z (the benchmark), 1 TENO6-A")
    ap.add_argument("--thinc", type=int, choices=[0, 1], default=0,
                    help="five-equation model: THINC interface capturing (1) or not (0, the benchmark)")
    ap.add_argument("--visc-order", type=int, choices=[4, 6], default=4,
                    help="central viscous stencils of the NS model: 4 (fused, the benchmark) or 6 "
                         "(separate passes; timed per fixed-dt step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one device copy of known size first (for HBM counter scaling)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the serving benchmark (0: skip it)")
    ap.add_argument("--serve-fill", type=int, default=768,
                    help="a request joins the running batch while the batch has fewer stage workgroups than "
                         "this (0: whenever a slot and memory are free); 768 = the FP32 stage workgroups resident "
                         "on 256 CUs at once")
    ap.add_argument("--serve-only", action="store_true", help="run the serving benchmark alone and print its JSON")
    ap.add_argument("--serve-eager", action="store_true", help="batched steps without graph replay")
    ap.add_argument("--serve-backlog", type=int, default=8,
                    help="srpt: beyond this many resident or queued requests every resident request steps "
                         "(0: keep the fill budget at any load)")
    ap.add_argument("--serve-policy", choices=["srpt", "fcfs"], default="srpt",
                    help="srpt: each step advances the resident requests with the least remaining work that fit "
                         "the fill budget; fcfs: requests join in arrival order and stay until done")
    ap.add_argument("--serve-protect-oldest", action="store_true",
                    help="srpt: step the oldest resident request in every step (shorter tail, longer median)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-max-batch", type=int, default=32)
    ap.add_argument("--serve-pool-gib", type=float, default=12.0)
    ap.add_argument("--serve-low-rate", type=float, default=20.0, help="arrival rate of the second stream")
    ap.add_argument("--serve-low-requests", type=int, default=200, help="requests of the second stream (0: skip)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiation benchmark")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (--gpus 1); several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2402_05193_amd import solver as S
    from paper_2402_05193_amd import workloads as WL

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.serve_only:
        res = run_serving(args.serve_requests, args.serve_rate, args.serve_max_batch, args.serve_pool_gib,
                          low_rate=args.serve_low_rate, low_n=args.serve_low_requests,
                          fill=args.serve_fill if args.serve_fill > 0 else None, use_graph=not args.serve_eager,
                          policy=args.serve_policy, backlog=args.serve_backlog if args.serve_backlog > 0 else None,
                          protect_oldest=args.serve_protect_oldest)
        print(json.dumps({"serving": res}), flush=True)
        return
    model = {"ns": S.NS, "euler": S.EULER, "dim": S.DIM}[args.model]
    dtype = S.F64 if args.dtype == "f64" else S.F32
    if model == S.DIM:
        case = WL.shock_bubble(2 * args.n if args.n < 256 else 256, args.n // 2 if args.n < 256 else 128,
                               args.n // 2 if args.n < 256 else 128, with_field=False)
        cfg = S.config_from_case(case, dtype=dtype, cfl=0.5, recon=args.recon, scheme=args.scheme,
                                     visc_order=args.visc_order if model == S.NS else 0, thinc=args.thinc)
        rho2, u2, p2 = case.meta["post_shock"]
        H = case.meta["H"]
        params = [0.060, 0.090, H / 2, H / 2, 0.25 * H, WL.ALPHA_EPS, rho2, u2, p2, 1.2041, 101325.0, 0.1660]
        case_id = S.CASE_SBI
        workload = (f"DIM shock-bubble Ma 1.22 air/He {cfg.nx}x{cfg.ny}x{cfg.nz}, limiters on, CFL 0.5"
                    f"{', characteristic reconstruction' if args.recon else ''}"
                    f"{', TENO6-A' if args.scheme else ''}{', THINC' if args.thinc else ''}")
    else:
        case = WL.taylor_green(args.n, viscous=(model == S.NS), with_field=False)
        cfg = S.config_from_case(case, dtype=dtype, cfl=0.5, recon=args.recon, scheme=args.scheme,
                                     visc_order=args.visc_order if model == S.NS else 0)
        params = [0.1, 1.0, 1e-3]
        case_id = S.CASE_TGV
        workload = (f"{'NS' if model == S.NS else 'Euler'} Taylor-Green vortex Ma 0.1"
                    f"{' Re 1600 Pr 0.72' if model == S.NS else ''} periodic {args.n}^3, CFL 0.5"
                    f"{', characteristic reconstruction' if args.recon else ''}"
                    f"{', TENO6-A' if args.scheme else ''}"
                    f"{', 6th-order viscous fluxes' if cfg.visc_order == 6 else ''}")

    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {nbytes} bytes read + {nbytes} bytes written", flush=True)
        del a, b

    U = S.empty_state(cfg, dev)
    S.init_state(cfg, case_id, params, U, seed=2402)
    A = torch.empty_like(U)
    B = torch.empty_like(U)
    ws = S.workspace(cfg, dev)
    dt_dev = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(events=None):
        if cfg.visc_order == 6:
            # sixth-order viscous passes + stage, three times, at the first step's dt
            if events is not None:
                events[0][0].record(stream)
            S.rk3_step(cfg, U, dt_fixed, ws)
            if events is not None:
                events[0][1].record(stream)
                for k in (1, 2):
                    events[k][0].record(stream)
                    events[k][1].record(stream)
            return
        # stage 1, stage 2, stage 3 fused with the CFL reduction that yields the next dt
        for k in range(3):
            if events is not None:
                events[k][0].record(stream)
            if k == 0:
                S.rk3_stage(cfg, 1, U, U, A, 0.0, dt_dev)
            elif k == 1:
                S.rk3_stage(cfg, 2, U, A, B, 0.0, dt_dev)
            else:
                S.rk3_stage3_cfl(cfg, U, B, U, dt_dev, dt_dev, ws)
            if events is not None:
                events[k][1].record(stream)

    S.compute_dt(cfg, U, dt_dev, ws)
    dt_fixed = float(dt_dev.item())
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(3)]
           for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for s in range(args.steps):
        step(evs[s])
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    stage_ms = [[evs[s][k][0].elapsed_time(evs[s][k][1]) for s in range(args.steps)] for k in range(3)]
    mean_stage_ms = sum(sum(x) for x in stage_ms) / (3 * args.steps)
    ncell = cfg.ncells
    value = ncell * 3 * args.steps / (ms_total * 1e-3)

    es = 8 if dtype == S.F64 else 4
    fpc = flops_per_cell(model, args.recon, args.scheme, cfg.visc_order)
    flops_launch = fpc * ncell
    achieved_tflops = flops_launch / (mean_stage_ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if dtype == S.F64 else PEAK_FP32_TFLOPS
    alg_bytes = sum(bytes_per_cell(cfg.ncomp, es, k + 1) for k in range(3)) / 3 * ncell
    hbm_gbs = alg_bytes / (mean_stage_ms * 1e-3) / 1e9

    finite = bool(torch.isfinite(U).all().item())
    # a device copy of 1 GiB timed like the stages: the HBM rate a streaming kernel attains here
    cbuf = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    cdst = torch.empty_like(cbuf)
    cdst.copy_(cbuf)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        cdst.copy_(cbuf)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * cbuf.numel() * 8 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del cbuf, cdst
    workload_key = (f"{args.model}-{args.dtype}-{args.n}" + ("-char" if args.recon else "")
                    + ("-teno" if args.scheme else "") + ("-v6" if cfg.visc_order == 6 else "")
                    + ("-thinc" if args.thinc else ""))
    # the stage instantiation this configuration runs, where it is one of the two profiled ones
    # (NS with the limiters off, the five-equation model with them on: positivity -1 selects
    # on for that model only); its fingerprint does not depend on the grid
    limiters_on = cfg.positivity == 1 or (cfg.positivity < 0 and model == S.DIM)
    kernel_symbol = None
    if workload_key.count("-") == 2 and limiters_on == (model == S.DIM):
        kernel_symbol = {"ns-f64": WORKLOAD_KERNELS["ns-f64-256"],
                         "dim-f64": WORKLOAD_KERNELS["dim-f64-256"]}.get(workload_key.rsplit("-", 1)[0])
    traffic = measured_traffic(workload_key) if kernel_symbol else None
    valu_per_cell = measured_valu_insts_per_cell(workload_key) if kernel_symbol else None
    t_stage = mean_stage_ms * 1e-3
    t_alu = flops_launch / (peak * 1e12)
    t_hbm = alg_bytes / (PEAK_HBM_GBS * 1e9)
    out = {
        "metric": "cell-updates/s + % HBM roofline (RK3 stage, 256^3); batched p50/p99 latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": None,             # one GPU: no scaling statement
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded analytic initial condition generated on the device)",
        "config": {"workload": workload, "cells": ncell, "ncomp": cfg.ncomp,
                   "counted_per": "RK stage (3 per step); stage 3 also reduces the next CFL time step"},
        "cell_steps_per_s": ncell * args.steps / (ms_total * 1e-3),
        "stage_ms": {"mean": mean_stage_ms, "stage1": sum(stage_ms[0]) / args.steps,
                     "stage2": sum(stage_ms[1]) / args.steps, "stage3": sum(stage_ms[2]) / args.steps},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved_tflops / peak, "traffic": traffic,
                     "kernel": "stage_kernel", "flops_per_cell": fpc,
                     "kernel_fingerprint": stage_kernel_hash(kernel_symbol) if kernel_symbol else None,
                     # max(t_HBM, t_ALU) / t over the algorithmic bytes and operations: the
                     # fraction of the attainable roofline, and the resource that sets it
                     "attainable_frac": max(t_alu, t_hbm) / t_stage,
                     "binding": "alu" if t_alu >= t_hbm else "hbm",
                     # VALU lane-instructions the kernel issues (committed counters of this
                     # kernel and workload) over the issue rate: the fraction of VALU issue
                     "valu_insts_per_cell": valu_per_cell,
                     "valu_issue_frac": (valu_per_cell * ncell / PEAK_VALU_LANE_INSTS / t_stage)
                                        if valu_per_cell else None},
        "hbm_roofline": {"achieved": hbm_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": hbm_gbs / PEAK_HBM_GBS, "bytes_per_cell_mean": alg_bytes / ncell,
                         "measured_copy_gbs": copy_gbs, "frac_of_copy": hbm_gbs / copy_gbs,
                         "traffic_gbs": (traffic / (mean_stage_ms * 1e-3) / 1e9) if traffic else None},
        "wall_s": wall,
        "state_finite": finite,
    }
    del U, A, B, ws
    torch.cuda.empty_cache()
    if args.serve_requests > 0:
        out["serving"] = run_serving(args.serve_requests, args.serve_rate, args.serve_max_batch,
                                     args.serve_pool_gib, low_rate=args.serve_low_rate,
                                     low_n=args.serve_low_requests,
                                     fill=args.serve_fill if args.serve_fill > 0 else None,
                                     use_graph=not args.serve_eager, policy=args.serve_policy,
                                     backlog=args.serve_backlog if args.serve_backlog > 0 else None,
                                     protect_oldest=args.serve_protect_oldest)
    if not args.no_adjoint:
        out["adjoint"] = run_adjoint_bench()
        print(f"[bench] adjoint: {json.dumps(out['adjoint'])}", flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = run_oracle_baseline(args.n, model)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
