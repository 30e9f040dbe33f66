"""Benchmark of the VMC hot path on one MI355X.

One step = one full pass of the hot path over one batch of synthetic input:
  Metropolis sampling (sweeps with cached hidden angles) + local energies of every
  sample + SR step (log-derivative products O v / O^dagger u inside an FP64 CG solve of
  (S + lambda I) x = F, then the parameter update).
Default workload: 1D spin-1/2 Heisenberg ring, N = 40, periodic, zero magnetisation via
nearest-neighbour exchange moves, Marshall-rotated; complex RBM with FP32 contractions,
alpha = 2 (80 hidden units), parameters N(0, 0.01^2) from seed 1234; 1024 chains x 200
sweeps = 204,800 samples per step; SR diagonal shift 0.01, learning rate 0.01, CG
tolerance 1e-8.

Prints one JSON line. value = samples per second of whole steps (sampling + local
energies + SR). Extra fields: the sampling-only rate, SR iterations per second, CG
iterations, the roofline of the dominant kernel, and the FP64 oracle timed on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

PEAK_FP32_VALU = 157.3e12
PEAK_FP32_MFMA = 157.3e12
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12

WORKLOADS = {
    "heisenberg1d_n40_cplx_fp32_alpha2": dict(L=40, ndim=1, diag=False, ham=1, J=(1.0, 0.0), h=0.0,
                                             marshall=True, move=1, cplx=True, prec=1, alpha=2,
                                             chains=1024, sweeps=200, lr=0.01, shift=0.01,
                                             cg_tol=1e-8, cg_maxiter=2000),
    "tfim1d_n10_real_fp64_alpha1": dict(L=10, ndim=1, diag=False, ham=0, J=(1.0, 0.0), h=1.0,
                                       marshall=False, move=0, cplx=False, prec=0, alpha=1,
                                       chains=16, sweeps=1000, lr=0.01, shift=0.01,
                                       cg_tol=1e-8, cg_maxiter=2000),
    # 10x10 J1-J2 (J2 = 0.5), Marshall-rotated, exchange moves, complex RBM alpha = 4:
    # 4096 chains x 2 sweeps = 8192 samples per step
    "j1j2_10x10_cplx_fp32_alpha4": dict(L=10, ndim=2, diag=True, ham=1, J=(1.0, 0.5), h=0.0,
                                        marshall=True, move=1, cplx=True, prec=1, alpha=4,
                                        chains=4096, sweeps=2, lr=0.01, shift=0.01,
                                        cg_tol=1e-8, cg_maxiter=500),
    "j1j2_10x10_cplx_bf16_alpha4": dict(L=10, ndim=2, diag=True, ham=1, J=(1.0, 0.5), h=0.0,
                                        marshall=True, move=1, cplx=True, prec=2, alpha=4,
                                        chains=4096, sweeps=2, lr=0.01, shift=0.01,
                                        cg_tol=1e-8, cg_maxiter=500),
    # 16x16 Heisenberg, complex RBM alpha = 8 (2048 hidden units), BF16 form:
    # 8192 chains x 1 sweep = 8192 samples per step
    "heis16x16_cplx_bf16_alpha8": dict(L=16, ndim=2, diag=False, ham=1, J=(1.0, 0.0), h=0.0,
                                       marshall=True, move=1, cplx=True, prec=2, alpha=8,
                                       chains=8192, sweeps=1, lr=0.01, shift=0.01,
                                       cg_tol=1e-8, cg_maxiter=500),
}


def cpu_baseline(w, N, M, seconds=15.0):
    """The FP64 oracle (plain numpy, unmodified) on a bounded sample of the same workload:
    a subset of the chains for a few sweeps, their local energies and one SR step."""
    import synth
    from oracle import hamiltonian as oh, lattice as ol, sampler as osamp, sr as osr
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = 1
    ob, osub = ol.hypercube(w["L"], w["ndim"], with_diagonals=w["diag"])
    om = oh.Model(N, M, ob, ham=w["ham"], J=w["J"], h=w["h"], marshall=w["marshall"],
                  sublattice=osub, move=w["move"], is_complex=w["cplx"])
    p = synth.rbm_params(N, M, w["cplx"], sigma=0.01, seed=1234)
    P = N + M + N * M
    # the oracle's SR forms S explicitly ([P, P]); beyond a few thousand parameters that
    # does not fit, and the baseline then covers sampling and local energies only
    with_sr = P <= 5000
    chains, sweeps = (64, 4) if N <= 64 else (16, 1)
    t0 = time.perf_counter()
    init = osamp.init_chains(om, chains, seed=1234)
    total_samples = 0
    while True:
        smp, init, _ = osamp.sample(om, p, init, sweeps, 0, seed=1234, counter=total_samples)
        flat = smp.reshape(-1, N)
        el = oh.local_energy(om, p, flat)
        if with_sr:
            osr.sr_step(om, p, flat, el, w["lr"], w["shift"], w["cg_tol"], w["cg_maxiter"])
        total_samples += flat.shape[0]
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    what = "local energies and one SR step" if with_sr else "local energies (no SR: the dense S of %d parameters does not fit)" % P
    return {"value": total_samples / dt, "unit": "samples/s", "cores": int(cores), "kind": "oracle",
            "sample": "%d chains x %d sweeps per pass, %s per pass, %d passes in %.1f s"
                      % (chains, sweeps, what, total_samples // (chains * sweeps), dt)}


def sv_flops(n, N, M, cplx):
    """Algorithmic flops of one S v product from cached tanh(theta) (n samples): z = sigma V
    (n x N x M, real spins times a real or complex direction), y = sum_j T (v_b + z) + sigma
    v_a, w = conj(T) y, O^dagger y = (w^T sigma, sum_s w, sigma^T y). Complex: 8nNM + 16nM +
    4nN; real: 4nNM + 6nM + 4nN."""
    if cplx:
        return 8.0 * n * N * M + 16.0 * n * M + 4.0 * n * N
    return 4.0 * n * N * M + 6.0 * n * M + 4.0 * n * N


def sv_bytes(n, N, M, cplx, masks):
    """Algorithmic HBM bytes of one S v product from cached tanh(theta): the T rows (n M
    values of 4 B, 8 B complex), the spins (one 8-byte mask per sample for the plane-split
    kernel, else n N int8), the direction in and the product out (P values in double)."""
    es = 8 if cplx else 4
    P = N + M + N * M
    spins = 8.0 * n if masks else float(n) * N
    return float(n) * M * es + spins + 2.0 * P * (16 if cplx else 8)


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, if one exists for the current kernel sources (the summary
    records a hash of them); None otherwise."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    try:
        srcs = fields["sources"].split()
        h = hashlib.sha256()
        for name in srcs:
            with open(os.path.join(ROOT, name), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != fields["sources_sha256"]:
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def copy_probe(torch, dev, mib=1024, reps=3):
    """A plain device-to-device copy of known size, for calibrating the FETCH_SIZE and
    WRITE_SIZE counters (each should read `mib` MiB per copy)."""
    a = torch.empty(mib << 20, dtype=torch.uint8, device=dev).fill_(1)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy probe: %d copies of %d MiB" % (reps, mib))


# batches of independent models: 64 periodic TFIM rings, N uniform in [16, 128], h uniform in
# [0.5, 1.5] (numpy PCG64, seed 1234), real FP32 RBM alpha = 2 each, 256 chains x 4 sweeps
# per ring per step
BATCH_WORKLOADS = {
    "tfim1d_batch64_n16to128_real_fp32_alpha2": dict(K=64, Nmin=16, Nmax=128, hmin=0.5, hmax=1.5,
                                                     alpha=2, chains=256, sweeps=4, prec=1,
                                                     lr=0.01, shift=0.01, cg_tol=1e-8,
                                                     cg_maxiter=500),
}


def batch_instances(w):
    rng = np.random.default_rng(1234)
    Ns = rng.integers(w["Nmin"], w["Nmax"] + 1, size=w["K"])
    hs = rng.uniform(w["hmin"], w["hmax"], size=w["K"])
    return [int(x) for x in Ns], [float(x) for x in hs]


def batch_cpu_baseline(w, seconds=15.0):
    """The FP64 oracle on a bounded sample of the batch: the first 8 rings, 16 chains x 4
    sweeps each, their local energies, and one SR step where the ring's dense S fits."""
    import synth
    from oracle import hamiltonian as oh, lattice as ol, sampler as osamp, sr as osr
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = 1
    Ns, hs = batch_instances(w)
    t0 = time.perf_counter()
    total, passes = 0, 0
    while time.perf_counter() - t0 < seconds:
        for k in range(8):
            N, M = Ns[k], w["alpha"] * Ns[k]
            ob, _ = ol.hypercube(N, 1)
            om = oh.Model(N, M, ob, ham=oh.TFIM, J=(1.0, 0.0), h=hs[k], move=oh.MOVE_FLIP)
            p = synth.rbm_params(N, M, False, sigma=0.01, seed=1234 + k)
            init = osamp.init_chains(om, 16, seed=1234 ^ k)
            smp, _, _ = osamp.sample(om, p, init, 4, 0, seed=1234 ^ k, counter=0)
            flat = smp.reshape(-1, N)
            el = oh.local_energy(om, p, flat)
            if N + M + N * M <= 5000:
                osr.sr_step(om, p, flat, el, w["lr"], w["shift"], w["cg_tol"], w["cg_maxiter"])
            total += flat.shape[0]
        passes += 1
    dt = time.perf_counter() - t0
    return {"value": total / dt, "unit": "samples/s", "cores": int(cores), "kind": "oracle",
            "sample": "first 8 rings of the batch, 16 chains x 4 sweeps each, local energies, and "
                      "one SR step for rings with at most 5000 parameters; %d passes in %.1f s"
                      % (passes, dt)}


def bench_batch(args, nqs, synth, torch, name):
    w = BATCH_WORKLOADS[name]
    dev = torch.device("cuda:0")
    Ns, hs = batch_instances(w)
    specs = []
    for N, h in zip(Ns, hs):
        bonds, sub = nqs.nqs_hypercube(N, 1)
        specs.append(dict(n_sites=N, n_hidden=w["alpha"] * N, bonds=bonds, ham=nqs.TFIM,
                          J=(1.0, 0.0), h=h, move=nqs.MOVE_FLIP, is_complex=False, prec=w["prec"]))
    b = nqs.Batch(specs)
    params = torch.from_numpy(np.concatenate(
        [synth.rbm_params(N, w["alpha"] * N, False, sigma=0.01, seed=1234 + k).astype(np.float32)
         for k, N in enumerate(Ns)])).to(dev)
    C, S = w["chains"], w["sweeps"]
    nch = [C] * w["K"]
    ns = [C * S] * w["K"]
    spins = sum(C * N for N in Ns)
    chains = torch.empty(spins, dtype=torch.int8, device=dev)
    b.chain_init(chains, nch, seed=1234)
    samples = torch.empty(S * spins, dtype=torch.int8, device=dev)
    eloc = torch.empty(S * C * w["K"], dtype=torch.float64, device=dev)
    ws = torch.empty(b.sr_workspace_bytes(ns), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    counter = [0]

    def step(discard):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.sample(params, chains, nch, S, discard, seed=1234, counter=counter[0], samples=samples,
                 eloc=eloc)
        e1.record(stream)
        counter[0] += S + discard
        infos = b.sr_step(params, samples, eloc, ns, w["lr"], w["shift"], w["cg_tol"],
                          w["cg_maxiter"], workspace=ws)
        return infos, (e0, e1)

    for k in range(args.warmup):
        infos, _ = step(10 if k == 0 else 0)
        log("warmup step %d: max cg_iters %d" % (k, max(i["cg_iters"] for i in infos)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs, iters = [], []
    for k in range(args.steps):
        infos, ev = step(0)
        evs.append(ev)
        iters.append(max(i["cg_iters"] for i in infos))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    samp_ms = sum(a.elapsed_time(c) for a, c in evs) / args.steps
    n_samp = C * S * w["K"]
    flops = float(sum(C * S * N * (w["alpha"] * N) * 4 for N in Ns))
    ach = flops / (samp_ms * 1e-3)
    out = {
        "metric": "samples/s (sweep+E_loc+O_k) and SR iters/s, BF16/FP32 vs FP64 at fixed dE",
        "value": n_samp / (ms_per_step * 1e-3), "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "instances": w["K"], "n_sites_min": min(Ns),
                   "n_sites_max": max(Ns), "chains_per_instance": C, "sweeps_per_step": S,
                   "samples_per_step": n_samp, "cg_tol": w["cg_tol"]},
        "sr_iters_per_s": 1e3 / ms_per_step,
        "phase_ms": {"sample_and_eloc": samp_ms, "sr_step": ms_per_step - samp_ms},
        "cg_iters_max_mean": float(np.mean(iters)),
        "roofline": {"kernel": "batched sweep with fused local energies (one launch)",
                     "bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": ach / PEAK_FP32_VALU, "traffic": None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


# exact ground energies of the workloads (Pauli units): Bethe ansatz for the 40-site
# Heisenberg ring, free-fermion closed form for the 10-site TFIM ring
E_REF = {"heisenberg1d_n40_cplx_fp32_alpha2": -70.98609115333286,
         "tfim1d_n10_real_fp64_alpha1": -12.784906442999324}
FORM_NAMES = {0: "fp64", 1: "fp32", 2: "bf16"}


def run_form(nqs, synth, torch, w, prec, iters):
    """SR trajectory of the workload in one precision form from the common start
    (parameters N(0, 0.01^2) from seed 1234, chains from seed 1234): per iteration one
    sampling call and one SR step; returns per-iteration energies and wall times."""
    dev = torch.device("cuda:0")
    N = w["L"] ** w["ndim"]
    M = w["alpha"] * N
    C, S = w["chains"], w["sweeps"]
    bonds, sub = nqs.nqs_hypercube(w["L"], w["ndim"], w["diag"])
    model = nqs.Model(N, M, bonds, ham=w["ham"], J=w["J"], h=w["h"], marshall=w["marshall"],
                      sublattice=sub, move=w["move"], is_complex=w["cplx"], prec=prec)
    p = synth.rbm_params(N, M, w["cplx"], sigma=0.01, seed=1234)
    params = torch.from_numpy(p).to(dev).to(model.param_dtype)
    chains = torch.empty((C, N), dtype=torch.int8, device=dev)
    model.chain_init(chains, seed=1234)
    samples = torch.empty((S, C, N), dtype=torch.int8, device=dev)
    eloc = torch.empty(S * C, dtype=model.value_dtype, device=dev)
    ws = torch.empty(model.sr_workspace_bytes(S * C), dtype=torch.uint8, device=dev)
    model.autotune(params, chains.repeat(S, 1), workspace=ws)
    energies, walls = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    counter = 0
    for k in range(iters):
        discard = max(10, S // 10) if k == 0 else 0
        model.sample(params, chains, S, discard, seed=1234, counter=counter, samples=samples,
                     eloc=eloc)
        counter += S + discard
        info = model.sr_step(params, samples.view(S * C, N), eloc, w["lr"], w["shift"],
                             w["cg_tol"], w["cg_maxiter"], workspace=ws)
        torch.cuda.synchronize()
        energies.append(info["energy_re"])
        walls.append(time.perf_counter() - t0)
    return energies, walls, S * C


def compare_forms(nqs, synth, torch, w, workload, iters):
    """The same SR trajectory in the FP64, FP32 and BF16 forms: rates, and the time each
    form needs to reach the energy error that all of them reach (dE = relative error of
    the 5-iteration running mean of the energy against the exact ground energy)."""
    out, runs = {}, {}
    for prec in (0, 1, 2):
        name = FORM_NAMES[prec]
        log("forms: %s, %d SR iterations" % (name, iters))
        energies, walls, n = run_form(nqs, synth, torch, w, prec, iters)
        runs[name] = ([np.mean(energies[max(0, k - 4):k + 1]) for k in range(len(energies))],
                      walls, n)
    # exact ground energy where one is known, else the FP64 form's final energy
    e_ref = E_REF.get(workload, float(runs["fp64"][0][-1]))
    curves = {}
    for name, (sm, walls, n) in runs.items():
        de = [abs(e - e_ref) / abs(e_ref) for e in sm]
        steady = (walls[-1] - walls[0]) / max(1, len(walls) - 1)   # excludes the burn-in call
        curves[name] = (de, walls)
        energies = sm
        out[name] = {"ms_per_iter": 1e3 * steady, "samples_per_s": n / steady,
                     "sr_iters_per_s": 1.0 / steady, "dE_final": de[-1],
                     "energy_final": float(energies[-1])}
    target = max(v["dE_final"] for v in out.values())
    if target == 0.0:
        target = 1e-12
    for name, (de, walls) in curves.items():
        k = next(i for i, d in enumerate(de) if d <= target)
        out[name]["iters_to_dE"] = k + 1
        out[name]["time_to_dE_s"] = walls[k]
    return {"dE_target": target, "e_ref": e_ref, "e_ref_kind": "exact" if workload in E_REF
            else "fp64 form, final", "iters": iters, "forms": out}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="heisenberg1d_n40_cplx_fp32_alpha2",
                    choices=list(WORKLOADS) + list(BATCH_WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--sv-pairs", type=int, default=0, choices=[0, 2, 4],
                    help="fixed S v kernel shape instead of the autotuner's choice")
    ap.add_argument("--forms-iters", type=int, default=40,
                    help="SR iterations per precision form in the FP64/FP32/BF16 comparison "
                         "(0 = skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the multi-GPU path (chains sharded across GPUs, "
              "one all-reduce of P values per CG iteration) is not built.", file=sys.stderr)
        sys.exit(2)

    log("importing torch")
    import torch
    import paper_1904_00031_amd as nqs
    import synth

    nqs.load()
    if args.copy_probe:
        copy_probe(torch, torch.device("cuda:0"))
    log("library loaded, building workload " + args.workload)
    if args.workload in BATCH_WORKLOADS:
        return bench_batch(args, nqs, synth, torch, args.workload)
    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    N = w["L"] ** w["ndim"]
    M = w["alpha"] * N
    C, S = w["chains"], w["sweeps"]
    bonds, sub = nqs.nqs_hypercube(w["L"], w["ndim"], w["diag"])
    model = nqs.Model(N, M, bonds, ham=w["ham"], J=w["J"], h=w["h"], marshall=w["marshall"],
                      sublattice=sub, move=w["move"], is_complex=w["cplx"], prec=w["prec"])
    p = synth.rbm_params(N, M, w["cplx"], sigma=0.01, seed=1234,
                         dtype=None if w["prec"] == 0 else (np.complex64 if w["cplx"] else np.float32))
    params = torch.from_numpy(p).to(dev)
    chains = torch.empty((C, N), dtype=torch.int8, device=dev)
    model.chain_init(chains, seed=1234)
    samples = torch.empty((S, C, N), dtype=torch.int8, device=dev)
    eloc = torch.empty(S * C, dtype=model.value_dtype, device=dev)
    nacc = torch.zeros(C, dtype=torch.int64, device=dev)
    ws = torch.empty(model.sr_workspace_bytes(S * C), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    counter = [0]

    def step(discard, times):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        model.sample(params, chains, S, discard, seed=1234, counter=counter[0], samples=samples,
                     n_accepted=nacc, eloc=eloc)
        counter[0] += S + discard
        e1.record(stream)
        info = model.sr_step(params, samples.view(S * C, N), eloc, w["lr"], w["shift"],
                             w["cg_tol"], w["cg_maxiter"], workspace=ws)
        e2.record(stream)
        if times is not None:
            times.append((e0, e1, e2, info))
        return info

    # pick the S v kernel shape for this model and sample count (timed on the
    # initial chains, before the timed region)
    if args.sv_pairs:
        model.set_sv_shape(args.sv_pairs)
        tune = {"fixed_pairs": args.sv_pairs}
    else:
        tune = model.autotune(params, chains.repeat(S, 1), workspace=ws)
    log("S v shape: %s" % tune)
    for k in range(args.warmup):
        info = step(max(10, S // 10) if k == 0 else 0, None)
        log("warmup step %d: E=%.8f cg_iters=%d" % (k, info["energy_re"], info["cg_iters"]))
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(0, times)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    samp_ms = sum(a.elapsed_time(b) for a, b, c, i in times) / args.steps
    sr_ms = sum(b.elapsed_time(c) for a, b, c, i in times) / args.steps
    cg = [i["cg_iters"] for a, b, c, i in times]
    energies = [i["energy_re"] for a, b, c, i in times]
    ms_per_step = wall * 1e3 / args.steps
    n_samp = S * C

    # live per-launch timing of the two parts that carry the work: the sampling call
    # (sweeps with fused local energies) and one S v product of the CG
    flat = samples.view(n_samp, N)
    reps = 5
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(reps):
        model.sample(params, chains, S, 0, seed=99, counter=10 ** 6, samples=samples, eloc=eloc)
    ev[1].record(stream)
    torch.cuda.synchronize()
    sweep_ms = ev[0].elapsed_time(ev[1]) / reps
    sv_reps = 20
    sv_ws = model.sr_prepare(params, flat, workspace=ws)
    gen = torch.Generator(device="cpu").manual_seed(5)
    v = torch.randn(model.n_params, dtype=model.value_dtype, generator=gen).to(dev)
    sv_out = torch.empty_like(v)
    model.sr_matvec(flat, sv_ws, v, w["shift"], out=sv_out)
    ev[0].record(stream)
    for _ in range(sv_reps):
        model.sr_matvec(flat, sv_ws, v, w["shift"], out=sv_out)
    ev[1].record(stream)
    torch.cuda.synchronize()
    mv_ms = ev[0].elapsed_time(ev[1]) / sv_reps

    sweep_flops = float(n_samp) * N * M * (12 if w["cplx"] else 4)
    mv_flops = sv_flops(n_samp, N, M, w["cplx"])
    share_sr = sr_ms / (samp_ms + sr_ms)
    # the plane-split product (complex, FP32 or BF16 form, N <= 63) runs its contractions
    # on the bf16 matrix cores with an exact three-part split (floor ~3x the flops at the
    # bf16 rate, below the time to stream T once): bounded by HBM. Other shapes run the
    # FP32 or FP64 16x16x4 MFMA and are reported against that peak.
    plane_split = w["cplx"] and w["prec"] != 0 and N <= 63
    if share_sr > 0.5 and plane_split:
        nbytes = sv_bytes(n_samp, N, M, w["cplx"], True)
        ach = nbytes / (mv_ms * 1e-3)
        roof = {"kernel": "S v product (direction tables, fused contraction, partial-sum "
                          "reduction, centring)", "bound": "hbm",
                "achieved": ach / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": ach / PEAK_HBM, "traffic": recorded_traffic("sv_product", args.workload),
                "algorithmic_bytes": nbytes,
                "fp32_equivalent_tflops": mv_flops / (mv_ms * 1e-3) / 1e12}
    elif share_sr > 0.5:
        peak = PEAK_FP64 if w["prec"] == 0 else PEAK_FP32_MFMA
        ach = mv_flops / (mv_ms * 1e-3)
        roof = {"kernel": "S v product (direction tables, fused contraction, partial-sum "
                          "reduction, centring)", "bound": "mfma",
                "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": recorded_traffic("sv_product", args.workload)}
    else:
        peak = PEAK_FP64 if w["prec"] == 0 else PEAK_FP32_VALU
        ach = sweep_flops / (sweep_ms * 1e-3)
        roof = {"kernel": "k_sweep", "bound": "alu", "achieved": ach / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": recorded_traffic("k_sweep", args.workload)}

    out = {
        "metric": "samples/s (sweep+E_loc+O_k) and SR iters/s, BF16/FP32 vs FP64 at fixed dE",
        "value": n_samp / (ms_per_step * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {0: "f64", 1: "f32", 2: "bf16"}[w["prec"]],
        "data": "synthetic",
        "config": {"workload": args.workload, "n_sites": N, "n_hidden": M, "chains": C,
                   "sweeps_per_step": S, "samples_per_step": n_samp, "cg_tol": w["cg_tol"],
                   "diag_shift": w["shift"], "lr": w["lr"]},
        "sr_iters_per_s": 1e3 / ms_per_step,
        "sampling_samples_per_s": n_samp / (samp_ms * 1e-3),
        "phase_ms": {"sample_and_eloc": samp_ms, "sr_step": sr_ms},
        "cg_iters_mean": float(np.mean(cg)),
        "energy_last": energies[-1],
        "kernel_ms": {"sample_call": sweep_ms, "sv_product": mv_ms},
        "sv_tuning": tune,
        "roofline": roof,
    }
    log("timed %d steps: %.2f ms/step" % (args.steps, ms_per_step))
    if args.forms_iters > 0:
        out["precision_forms"] = compare_forms(nqs, synth, torch, w, args.workload,
                                               args.forms_iters)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, N, M, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
