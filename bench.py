"""Benchmark of the VMC hot path on one MI355X.

One step = one full pass of the hot path over one batch of synthetic input:
  Metropolis sampling (sweeps with cached hidden angles) + local energies of every
  sample + SR step (log-derivative products O v / O^dagger u inside an FP64 CG solve of
  (S + lambda I) x = F, then the parameter update).

Headline workload (the largest single-GPU configuration): 2D Heisenberg antiferromagnet
on the 16 x 16 periodic square lattice, zero magnetisation via nearest-neighbour exchange
moves, Marshall-rotated; complex RBM with alpha = 8 (2048 hidden units) in the BF16 form
(weights rounded to bfloat16, float arithmetic, bfloat16 tanh(theta) in the Jacobian
contractions) with FP64 CG; parameters N(0, 0.01^2) from seed 1234; 8192 chains x 1 sweep
= 8192 samples per step; SR shift 0.01, lr 0.01, CG tolerance 1e-8, at most 500 products.

Prints one JSON line. value = samples per second of whole steps. Extra fields: phase
times, the roofline of the step's dominant kernel (measured live with HIP events on the
launch stream), the other workloads of the benchmark family (10-site TFIM, 40-site
Heisenberg ring, 10x10 J1-J2 in FP32 and BF16, the symmetric RBM, the batch of 64 TFIM
rings replayed from a captured graph, parallel tempering on the 6x6 J1-J2 lattice, a
two-layer feed-forward network on the 40-site ring, and supervised learning of a 20-site
target) with their own rooflines or rates, the FP64 / FP32 / BF16 forms of the 40-site
ring compared at a fixed energy error, and the FP64 oracle timed on the host.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

# MI355X peaks (AMD's published dense figures)
PEAK_FP32_VALU = 157.3e12
PEAK_FP32_MFMA = 157.3e12
PEAK_FP64 = 78.6e12
PEAK_BF16_MFMA = 2500e12
PEAK_HBM = 8.0e12

HEADLINE = "heis16x16_cplx_bf16_alpha8"
METRIC = "samples/s (sweep+E_loc+O_k) and SR iters/s, BF16/FP32 vs FP64 at fixed dE"

WORKLOADS = {
    # 16x16 Heisenberg, complex RBM alpha = 8 (2048 hidden units), BF16 form, FP64 CG
    "heis16x16_cplx_bf16_alpha8": dict(L=16, ndim=2, diag=False, ham=1, J=(1.0, 0.0), h=0.0,
                                       marshall=True, move=1, cplx=True, prec=2, alpha=8,
                                       chains=8192, sweeps=1, lr=0.01, shift=0.01,
                                       cg_tol=1e-8, cg_maxiter=500),
    # 1D Heisenberg ring, N = 40, complex FP32 RBM alpha = 2: 1024 chains x 200 sweeps
    "heisenberg1d_n40_cplx_fp32_alpha2": dict(L=40, ndim=1, diag=False, ham=1, J=(1.0, 0.0), h=0.0,
                                             marshall=True, move=1, cplx=True, prec=1, alpha=2,
                                             chains=1024, sweeps=200, lr=0.01, shift=0.01,
                                             cg_tol=1e-8, cg_maxiter=2000),
    # 1D TFIM ring, N = 10, real FP64 RBM alpha = 1: 16 chains x 1000 sweeps
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
    # the symmetric RBM (filters shared over the 256 translations) on the 16x16 lattice,
    # alpha = 8 (the same 2048 hidden units, 2057 parameters), BF16 form
    "heis16x16_symm_cplx_bf16_alpha8": dict(L=16, ndim=2, diag=False, ham=1, J=(1.0, 0.0), h=0.0,
                                            marshall=True, move=1, cplx=True, prec=2, alpha=8,
                                            chains=8192, sweeps=1, lr=0.01, shift=0.01,
                                            cg_tol=1e-8, cg_maxiter=500, symm=True),
}
EXTRA_SINGLE = ["heisenberg1d_n40_cplx_fp32_alpha2", "tfim1d_n10_real_fp64_alpha1",
                "j1j2_10x10_cplx_fp32_alpha4", "j1j2_10x10_cplx_bf16_alpha4",
                "heis16x16_symm_cplx_bf16_alpha8"]

# batches of independent models: 64 periodic TFIM rings, N uniform in [16, 128], h uniform in
# [0.5, 1.5] (numpy PCG64, seed 1234), real FP32 RBM alpha = 2 each, 256 chains x 4 sweeps
# per ring per step; the step (sampling + stream-ordered SR with at most 100 CG slots) is
# captured into one graph and replayed
BATCH_WORKLOADS = {
    "tfim1d_batch64_n16to128_real_fp32_alpha2": dict(K=64, Nmin=16, Nmax=128, hmin=0.5, hmax=1.5,
                                                     alpha=2, chains=256, sweeps=4, prec=1,
                                                     lr=0.01, shift=0.01, cg_tol=1e-8,
                                                     cg_maxiter=100),
}

# parallel tempering: 10x10 is beyond the tempered FP32 sweep (at most 256 hidden units),
# so the 6x6 J1-J2 lattice (J2 = 0.5), complex FP32 RBM alpha = 4, 2048 tempered chains of
# 4 replicas (beta = 1, 3/4, 1/2, 1/4), 4 recorded sweeps per step with local energies
PT_WORKLOAD = dict(name="j1j2_6x6_cplx_fp32_alpha4_pt4", L=6, ndim=2, diag=True, ham=1,
                   J=(1.0, 0.5), h=0.0, marshall=True, move=1, cplx=True, prec=1, alpha=4,
                   chains=2048, replicas=4, sweeps=4)

# the feed-forward network: 40-site Heisenberg ring, two dense layers 40 -> 80 -> 40 with
# ln cosh activations, complex FP32, parameters N(0, 0.01^2); 1024 chains x 20 sweeps per
# step, SR with shift 0.01, lr 0.01, CG tolerance 1e-8, at most 200 products
FF_WORKLOAD = dict(name="heisenberg1d_n40_cplx_fp32_ffnn80x40", L=40, ndim=1, diag=False, ham=1,
                   J=(1.0, 0.0), h=0.0, marshall=True, move=1, cplx=True, prec=1,
                   layers=[80, 40], acts=[0, 0], chains=1024, sweeps=20, lr=0.01, shift=0.01,
                   cg_tol=1e-8, cg_maxiter=200)

# supervised learning (Eq. 1, Eq. 2): a 20-site training set (all 2^20 configurations) whose
# target is a teacher RBM (20 hidden units, complex, N(0, 0.1^2), seed 7); student complex
# FP32 RBM with 40 hidden units, N(0, 0.01^2) from seed 1234; 16384 direct draws per step,
# SGD with lr 0.05
SUP_WORKLOAD = dict(name="supervised_n20_teacher_rbm_student_alpha2_fp32", N=20, M_teacher=20,
                    M=40, prec=1, batch=16384, lr=0.05)

GOLDEN = os.path.join(ROOT, "tests", "golden", "reference_energies.txt")


def golden(name):
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#") and line.split()[0] == name:
                return float(line.split()[1])
    raise KeyError(name)


# exact ground energies of the workloads (Pauli units): Bethe ansatz for the 40-site
# Heisenberg ring, free-fermion closed form for the 10-site TFIM ring
E_REF = {"heisenberg1d_n40_cplx_fp32_alpha2": "heis_ring_n40",
         "tfim1d_n10_real_fp64_alpha1": "tfim_n10_h1"}
FORM_NAMES = {0: "fp64", 1: "fp32", 2: "bf16"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return nproc, model


# ---- algorithmic work ------------------------------------------------------------------
def sweep_terms_flops(cplx):
    """Flops of one ratio term cosh(d) + tanh(theta) sinh(d) and its share of |ratio|^2:
    complex t S (6) and C - s t S (2), |term|^2 (3), product (1) = 12; real: 4."""
    return 12.0 if cplx else 4.0


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


def recorded_traffic(kernel, workload, real_move_fraction=None):
    """HBM bytes per launch of `kernel` on `workload` from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, if one exists for the current kernel sources (the summary
    records a hash of them); None otherwise. A sweep's record also holds the fraction of
    non-identity proposals of its run: the bytes are scaled to this run's fraction (the
    table rows are fetched per non-identity proposal)."""
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
        h = hashlib.sha256()
        for name in fields["sources"].split():
            with open(os.path.join(ROOT, name), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != fields["sources_sha256"]:
            return None
        b = float(fields["hbm_bytes_per_launch"])
        if real_move_fraction is not None and "real_move_fraction" in fields:
            b *= real_move_fraction / float(fields["real_move_fraction"])
        return b
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


# ---- one model ---------------------------------------------------------------------------
class Single:
    def __init__(self, nqs, synth, torch, name, prec=None):
        self.torch = torch
        self.name = name
        self.w = w = WORKLOADS[name]
        self.prec = w["prec"] if prec is None else prec
        self.dev = torch.device("cuda:0")
        self.N = N = w["L"] ** w["ndim"]
        self.M = M = w["alpha"] * N
        self.C, self.S = w["chains"], w["sweeps"]
        bonds, sub = nqs.nqs_hypercube(w["L"], w["ndim"], w["diag"])
        self.bonds0 = torch.from_numpy(np.asarray(bonds[0], dtype=np.int64)).to(self.dev)
        symm = nqs.nqs_hypercube_translations(w["L"], w["ndim"]) if w.get("symm") else None
        self.model = nqs.Model(N, M, bonds, ham=w["ham"], J=w["J"], h=w["h"],
                               marshall=w["marshall"], sublattice=sub, move=w["move"],
                               is_complex=w["cplx"], prec=self.prec, symm=symm)
        if symm is None:
            p = synth.rbm_params(N, M, w["cplx"], sigma=0.01, seed=1234)
        else:
            rng = np.random.default_rng(1234)
            P = self.model.n_params
            p = rng.normal(0.0, 0.01, P) + (1j * rng.normal(0.0, 0.01, P) if w["cplx"] else 0)
        self.params = torch.from_numpy(p).to(self.dev).to(self.model.param_dtype)
        self.chains = torch.empty((self.C, N), dtype=torch.int8, device=self.dev)
        self.model.chain_init(self.chains, seed=1234)
        self.samples = torch.empty((self.S, self.C, N), dtype=torch.int8, device=self.dev)
        self.eloc = torch.empty(self.S * self.C, dtype=self.model.value_dtype, device=self.dev)
        self.ws = torch.empty(self.model.sr_workspace_bytes(self.S * self.C), dtype=torch.uint8,
                              device=self.dev)
        self.stream = torch.cuda.current_stream()
        self.counter = 0

    def step(self, discard, times=None):
        torch, m, w = self.torch, self.model, self.w
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)] if times is not None else None
        if ev:
            ev[0].record(self.stream)
        m.sample(self.params, self.chains, self.S, discard, seed=1234, counter=self.counter,
                 samples=self.samples, eloc=self.eloc)
        self.counter += self.S + discard
        if ev:
            ev[1].record(self.stream)
        info = m.sr_step(self.params, self.samples.view(self.S * self.C, self.N), self.eloc,
                         w["lr"], w["shift"], w["cg_tol"], w["cg_maxiter"], workspace=self.ws,
                         n_chains=self.C)
        if ev:
            ev[2].record(self.stream)
            times.append((ev, info))
        return info

    def real_move_fraction(self):
        """Fraction of proposals that are not the identity: 1 for flips; for exchanges the
        fraction of color-0 bonds with opposite spins in the recorded samples."""
        if self.w["move"] == 0:
            return 1.0
        s = self.samples.view(-1, self.N)
        b = self.bonds0
        return float((s[:, b[:, 0]] != s[:, b[:, 1]]).float().mean().item())

    def fused_eloc(self):
        """Whether nqs_sample evaluates the local energies inside the sweep (at least 16
        chains per compute unit and at most 256 hidden units)."""
        cus = self.torch.cuda.get_device_properties(0).multi_processor_count
        return self.C >= 16 * cus and self.M <= 256

    def run(self, steps, warmup, tune=True):
        torch, m, w = self.torch, self.model, self.w
        nqs = sys.modules["paper_1904_00031_amd"]
        tuning = m.autotune(self.params, self.chains.repeat(self.S, 1), workspace=self.ws) \
            if tune else None
        for k in range(warmup):
            info = self.step(max(10, self.S // 10) if k == 0 else 0)
            log("%s warmup %d: E=%.6f +- %.2e cg_iters=%d" % (self.name, k, info["energy_re"],
                                                                info["energy_err"], info["cg_iters"]))
        torch.cuda.synchronize()
        # the sweep kernel of every timed step is bracketed by HIP events on its stream
        m.time_kernel(nqs.TIME_SWEEP)
        times, sweep_k = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step(0, times)          # the SR step synchronises the stream
            sweep_k.append(m.kernel_ms())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        m.time_kernel(nqs.TIME_NONE)
        samp_ms = sum(e[0].elapsed_time(e[1]) for e, _ in times) / steps
        sr_ms = sum(e[1].elapsed_time(e[2]) for e, _ in times) / steps
        infos = [i for _, i in times]
        ms_per_step = wall * 1e3 / steps
        n = self.S * self.C
        f_real = self.real_move_fraction()
        sweep_ms = float(np.mean(sweep_k))

        # after the timed region: the local-energy kernel and one S v product (the CG's
        # products replay from graphs), each bracketed by the library's events
        flat = self.samples.view(n, self.N)
        el2 = torch.empty_like(self.eloc)
        reps = 5
        m.time_kernel(nqs.TIME_ELOC)
        el_k = []
        for _ in range(reps):
            m.local_energy(self.params, flat, out=el2)
            el_k.append(m.kernel_ms())
        eloc_ms = float(np.mean(el_k[1:]))
        sv_ws = m.sr_prepare(self.params, flat, workspace=self.ws)
        gen = torch.Generator(device="cpu").manual_seed(5)
        v = torch.randn(m.n_params, dtype=m.value_dtype, generator=gen).to(self.dev)
        sv_out = torch.empty_like(v)
        # the product's kernels: the library's event pair around each of them (direction
        # tables, O v, O^dagger y or the fused product, reduction), per product
        m.time_kernel(nqs.TIME_SV)
        sv_pairs = []
        for _ in range(21):
            m.sr_matvec(flat, sv_ws, v, w["shift"], out=sv_out)
            sv_pairs.append(m.kernel_times())
        m.time_kernel(nqs.TIME_NONE)
        sv_pairs = np.array(sv_pairs[1:])
        pair_ms = sv_pairs.mean(axis=0)
        mv_ms = float(pair_ms.sum())
        cg_mean = float(np.mean([i["cg_iters"] for i in infos]))

        # roofline of the single kernel with the largest device time per step: the sweep,
        # the local energies (when not fused into the sweep), or one of the S v product's
        # kernels times the CG iterations per step (the product's kernels, each timed by
        # the library's event pair: direction tables, O v, O^dagger y or the fused product,
        # the reduction)
        cplx = w["cplx"]
        es = (16 if cplx else 8) if self.prec == 0 else (8 if cplx else 4)
        fused_sv = len(pair_ms) == 3
        share = {"sweep": sweep_ms}
        if not self.fused_eloc():
            share["eloc"] = eloc_ms
        if fused_sv:
            share["sv_fused"] = float(pair_ms[1]) * cg_mean
        else:
            share["jvp"] = float(pair_ms[1]) * cg_mean
            share["vjp"] = float(pair_ms[2]) * cg_mean
        dom = max(share, key=share.get)
        itiles = (self.N + 1 + 15) // 16
        if dom == "sweep" and self.prec != 0 and self.M > 256:
            # the wide sweep reads the two table rows (M values each) of every non-identity
            # proposal from global memory (16.8 MB of tables, no reuse across chains)
            nbytes = float(self.C) * self.S * self.N * f_real * 2 * self.M * es
            ach = nbytes / (sweep_ms * 1e-3)
            roof = {"kernel": "k_sweep_wide", "bound": "hbm", "achieved": ach / 1e9,
                    "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": ach / PEAK_HBM,
                    "traffic": recorded_traffic("k_sweep_wide", self.name, f_real),
                    "algorithmic_bytes": nbytes, "launch_ms": sweep_ms,
                    "real_move_fraction": f_real,
                    "ratio_term_tflops": float(self.C) * self.S * self.N * f_real * self.M *
                    sweep_terms_flops(cplx) / (sweep_ms * 1e-3) / 1e12}
        elif dom == "sweep":
            peak = PEAK_FP64 if self.prec == 0 else PEAK_FP32_VALU
            fl = float(self.C) * self.S * self.N * f_real * self.M * sweep_terms_flops(cplx)
            ach = fl / (sweep_ms * 1e-3)
            roof = {"kernel": "k_sweep", "bound": "alu", "achieved": ach / 1e12,
                    "peak": peak / 1e12, "unit": "TFLOP/s", "frac": ach / peak,
                    "traffic": recorded_traffic("k_sweep", self.name),
                    "algorithmic_flops": fl, "launch_ms": sweep_ms, "real_move_fraction": f_real}
        elif dom == "sv_fused" and cplx and self.prec != 0 and self.N <= 63:
            # the plane-split fused product streams the T rows (complex FP32, or bfloat16
            # pairs in the BF16 form) and spin masks once
            nbytes = float(n) * self.M * (4 if self.prec == 2 else 8) + 8.0 * n
            t = float(pair_ms[1])
            ach = nbytes / (t * 1e-3)
            roof = {"kernel": "k_svc", "bound": "hbm", "achieved": ach / 1e9,
                    "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": ach / PEAK_HBM,
                    "traffic": recorded_traffic("k_svc", self.name),
                    "algorithmic_bytes": nbytes, "launch_ms": t,
                    "fp32_equivalent_tflops": sv_flops(n, self.N, self.M, cplx) / (t * 1e-3) / 1e12}
        elif dom in ("jvp", "vjp", "sv_fused"):
            # contractions against the spin matrix: 4 n N M flops each side (complex), 2 n N M
            # (real). FP64 models run them on the FP64 matrix cores; the FP32 / BF16 forms on
            # the bf16 matrix cores with the float operand split exactly into three bf16
            # parts: VJP parts h, m in one 16x16x32 instruction and l in a second (4x the
            # flops), JVP three parts (3x). Those are reported against the bf16 peak by the
            # flops of the bf16 instructions issued, with the float-equivalent rate alongside
            t = float(pair_ms[1] if dom in ("jvp", "sv_fused") else pair_ms[2])
            side = (4.0 if cplx else 2.0) * n * self.N * self.M
            fl = 2 * side if dom == "sv_fused" else side
            name = {"jvp": "k_jvp32" if self.prec != 0 else "k_jvp",
                    "vjp": ("k_vjp_wide" if 5 <= itiles <= 17 else "k_vjp"),
                    "sv_fused": "k_sv"}[dom]
            if self.prec == 0:
                ach, peak, ifl = fl / (t * 1e-3), PEAK_FP64, fl
            else:
                mult = {"jvp": 3.0, "vjp": 4.0, "sv_fused": 3.5}[dom]
                ifl = mult * fl
                ach, peak = ifl / (t * 1e-3), PEAK_BF16_MFMA
            roof = {"kernel": name, "bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12,
                    "unit": "TFLOP/s", "frac": ach / peak,
                    "traffic": recorded_traffic(name, self.name),
                    "algorithmic_flops": ifl, "launch_ms": t}
            if self.prec != 0:
                roof["float_equivalent_flops"] = fl
                roof["float_equivalent_frac_of_fp32_matrix_peak"] = fl / (t * 1e-3) / PEAK_FP32_MFMA
        else:
            peak = PEAK_FP64 if self.prec == 0 else PEAK_FP32_VALU
            fl = float(n) * self.N * f_real * self.M * sweep_terms_flops(cplx)
            ach = fl / (eloc_ms * 1e-3)
            roof = {"kernel": "k_eloc_rows" if self.M > 256 else "local energy",
                    "bound": "alu", "achieved": ach / 1e12,
                    "peak": peak / 1e12, "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                    "algorithmic_flops": fl, "launch_ms": eloc_ms}
        # the whole S v product for reference (sum of its kernels' times)
        svf = sv_flops(n, self.N, self.M, cplx)
        roof["sv_product"] = {"ms": mv_ms, "kernel_ms": [float(x) for x in pair_ms],
                              "fp32_equivalent_tflops": svf / (mv_ms * 1e-3) / 1e12,
                              "frac_of_fp32_matrix_peak": svf / (mv_ms * 1e-3) / PEAK_FP32_MFMA}
        roof["step_share_ms"] = share
        return {
            "ms_per_step": ms_per_step, "samples_per_step": n,
            "value": n / (ms_per_step * 1e-3),
            "sr_iters_per_s": 1e3 / ms_per_step,
            "sampling_samples_per_s": n / (samp_ms * 1e-3),
            "phase_ms": {"sample_and_eloc": samp_ms, "sr_step": sr_ms},
            "kernel_ms": {"sweep": sweep_ms, "local_energy": eloc_ms, "sv_product": mv_ms},
            "cg_iters_mean": cg_mean, "real_move_fraction": f_real,
            "energy_last": infos[-1]["energy_re"], "energy_err_last": infos[-1]["energy_err"],
            "sv_tuning": tuning, "roofline": roof,
        }


# ---- batch of models, graph-captured step ------------------------------------------------
def bench_pt(nqs, synth, torch, steps, warmup):
    """Tempered sampling with local energies: recorded samples per second, the sweep
    kernel's roofline over every replica's proposals, exchange acceptance."""
    w = PT_WORKLOAD
    dev = torch.device("cuda:0")
    N = w["L"] ** w["ndim"]
    M = w["alpha"] * N
    C, R, S = w["chains"], w["replicas"], w["sweeps"]
    bonds, sub = nqs.nqs_hypercube(w["L"], w["ndim"], w["diag"])
    m = nqs.Model(N, M, bonds, ham=w["ham"], J=w["J"], h=w["h"], marshall=w["marshall"],
                  sublattice=sub, move=w["move"], is_complex=w["cplx"], prec=w["prec"])
    p = torch.from_numpy(synth.rbm_params(N, M, w["cplx"], sigma=0.01, seed=1234)).to(dev)
    p = p.to(m.param_dtype)
    ch = torch.empty((C * R, N), dtype=torch.int8, device=dev)
    m.chain_init(ch, seed=1234)
    reps = ch.view(C, R, N)
    tix = torch.arange(R, dtype=torch.int32, device=dev).repeat(C, 1).contiguous()
    samples = torch.empty((S, C, N), dtype=torch.int8, device=dev)
    eloc = torch.empty(S * C, dtype=m.value_dtype, device=dev)
    nsw = torch.zeros(C, dtype=torch.int64, device=dev)
    counter = 0
    for k in range(warmup):
        m.sample_pt(p, reps, tix, S, 10 if k == 0 else 0, seed=1234, counter=counter,
                    samples=samples, eloc=eloc, n_swaps=nsw)
        counter += S + (10 if k == 0 else 0)
    torch.cuda.synchronize()
    # exchange counts summed per chain on the device; the accumulation runs once before the
    # timed region so that loading its kernel is not timed
    swaps_dev = torch.zeros(C, dtype=torch.int64, device=dev)
    swaps_dev += nsw
    swaps_dev.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m.sample_pt(p, reps, tix, S, 0, seed=1234, counter=counter, samples=samples, eloc=eloc,
                    n_swaps=nsw)
        counter += S
        swaps_dev += nsw
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    swaps = int(swaps_dev.sum().item())
    # after the timed region: the tempered sweep kernel of a few more calls, each bracketed
    # by the library's event pair (waiting on it inside the timed loop would stall the host)
    m.time_kernel(nqs.TIME_SWEEP)
    sweep_k = []
    for _ in range(5):
        m.sample_pt(p, reps, tix, S, 0, seed=1234, counter=counter, samples=samples, eloc=eloc)
        counter += S
        sweep_k.append(m.kernel_ms())
    m.time_kernel(nqs.TIME_NONE)
    ms = wall * 1e3 / steps
    sweep_ms = float(np.mean(sweep_k))
    b = torch.from_numpy(np.asarray(bonds[0], dtype=np.int64)).to(dev)
    s = samples.view(-1, N)
    f_real = float((s[:, b[:, 0]] != s[:, b[:, 1]]).float().mean().item())
    fl = float(C) * R * S * N * f_real * M * sweep_terms_flops(w["cplx"])
    ach = fl / (sweep_ms * 1e-3)
    return {"workload": w["name"], "dtype": "f32", "ms_per_step": ms,
            "samples_per_step": S * C, "value": S * C / (ms * 1e-3), "unit": "samples/s",
            "replica_sweeps_per_s": C * R * S / (ms * 1e-3),
            "swap_acceptance": swaps / float(steps * S * C * (R - 1)),
            "energy_per_site": float(eloc.real.mean().item()) / N,
            "roofline": {"kernel": "k_sweep (tempered)", "bound": "alu", "achieved": ach / 1e12,
                         "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": ach / PEAK_FP32_VALU, "traffic": None,
                         "algorithmic_flops": fl, "launch_ms": sweep_ms,
                         "real_move_fraction": f_real}}


def ff_macs(layers, N, first=True):
    """Multiply-adds of one forward pass of the dense layers (from layer 0 or layer 1)."""
    w = [N] + list(layers)
    return sum(w[l] * w[l + 1] for l in range(0 if first else 1, len(layers)))


def bench_ffnn(nqs, synth, torch, steps, warmup):
    """The network's VMC step (sampling + local energies + SR): samples per second, phase
    and kernel times, and the roofline of the kernel that takes most of the step."""
    w = FF_WORKLOAD
    dev = torch.device("cuda:0")
    N = w["L"] ** w["ndim"]
    C, S = w["chains"], w["sweeps"]
    bonds, sub = nqs.nqs_hypercube(w["L"], w["ndim"], w["diag"])
    m = nqs.Model(N, w["layers"][0], bonds, ham=w["ham"], J=w["J"], h=w["h"],
                  marshall=w["marshall"], sublattice=sub, move=w["move"], is_complex=w["cplx"],
                  prec=w["prec"], layers=w["layers"], activations=w["acts"])
    rng = np.random.default_rng(1234)
    P = m.n_params
    p = rng.normal(0, 0.01, P) + 1j * rng.normal(0, 0.01, P)
    params = torch.from_numpy(p).to(dev).to(m.param_dtype)
    ch = torch.empty((C, N), dtype=torch.int8, device=dev)
    m.chain_init(ch, seed=1234)
    samples = torch.empty((S, C, N), dtype=torch.int8, device=dev)
    eloc = torch.empty(S * C, dtype=m.value_dtype, device=dev)
    ws = torch.empty(m.sr_workspace_bytes(S * C), dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream()
    counter = 0

    def step(discard, ev=None):
        nonlocal counter
        if ev:
            ev[0].record(st)
        m.sample(params, ch, S, discard, seed=1234, counter=counter, samples=samples, eloc=eloc)
        counter += S + discard
        if ev:
            ev[1].record(st)
        info = m.sr_step(params, samples.view(S * C, N), eloc, w["lr"], w["shift"], w["cg_tol"],
                         w["cg_maxiter"], workspace=ws, n_chains=C)
        if ev:
            ev[2].record(st)
        return info

    for k in range(warmup):
        step(10 if k == 0 else 0)
    torch.cuda.synchronize()
    m.time_kernel(nqs.TIME_SWEEP)
    evs, infos, sweep_k = [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        infos.append(step(0, ev))
        evs.append(ev)
        sweep_k.append(m.kernel_ms())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n = S * C
    flat = samples.view(n, N)
    m.time_kernel(nqs.TIME_ELOC)
    el_k = []
    for _ in range(4):
        m.local_energy(params, flat, out=torch.empty_like(eloc))
        el_k.append(m.kernel_ms())
    m.time_kernel(nqs.TIME_SV)
    gen = torch.Generator(device="cpu").manual_seed(5)
    v = torch.randn(P, dtype=m.value_dtype, generator=gen).to(dev)
    u = torch.randn(n, dtype=m.value_dtype, generator=gen).to(dev)
    sv_k = []
    for _ in range(6):
        m.log_psi_grad(params, flat, u=u, v=v)
        sv_k.append(m.kernel_ms())
    m.time_kernel(nqs.TIME_NONE)
    ms = wall * 1e3 / steps
    sweep_ms, eloc_ms, sv_ms = (float(np.mean(sweep_k)), float(np.mean(el_k[1:])),
                                float(np.mean(sv_k[1:])))
    cg_mean = float(np.mean([i["cg_iters"] for i in infos]))
    b = torch.from_numpy(np.asarray(bonds[0], dtype=np.int64)).to(dev)
    f_real = float((flat[:, b[:, 0]] != flat[:, b[:, 1]]).float().mean().item())
    cm = 8.0   # flops of a complex multiply-add
    later = ff_macs(w["layers"], N, first=False)
    per_prop = cm * later + 4.0 * 2 * w["layers"][0]   # later layers + two angle columns
    sweep_fl = float(C) * S * N * f_real * per_prop
    eloc_fl = float(n) * len(bonds[0]) * f_real * per_prop
    sv_fl = float(n) * 2 * cm * ff_macs(w["layers"], N)
    share = {"sweep": sweep_ms, "eloc": eloc_ms, "sv": sv_ms * cg_mean}
    dom = max(share, key=share.get)
    fl, kms, kname = {"sweep": (sweep_fl, sweep_ms, "k_ff_sweep"),
                      "eloc": (eloc_fl, eloc_ms, "k_ff_eloc"),
                      "sv": (sv_fl, sv_ms, "k_ff_prep_dir + k_ff_jvp + k_ff_vjp + "
                                          "k_ff_vjp_reduce")}[dom]
    ach = fl / (kms * 1e-3)
    return {"workload": w["name"], "dtype": "f32", "ms_per_step": ms, "samples_per_step": n,
            "value": n / (ms * 1e-3), "unit": "samples/s", "sr_iters_per_s": 1e3 / ms,
            "phase_ms": {"sample_and_eloc": float(np.mean([e[0].elapsed_time(e[1]) for e in evs])),
                         "sr_step": float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))},
            "kernel_ms": {"sweep": sweep_ms, "local_energy": eloc_ms, "jvp_plus_vjp": sv_ms},
            "cg_iters_mean": cg_mean, "energy_last": infos[-1]["energy_re"],
            "roofline": {"kernel": kname, "bound": "alu", "achieved": ach / 1e12,
                         "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": ach / PEAK_FP32_VALU, "traffic": None, "algorithmic_flops": fl,
                         "launch_ms": kms, "step_share_ms": share}}


def bench_supervised(nqs, synth, torch, steps, warmup):
    """Supervised steps (direct draws from |t|^2 + the overlap step): steps and draws per
    second, the loss before and after."""
    w = SUP_WORKLOAD
    dev = torch.device("cuda:0")
    N, M = w["N"], w["M"]
    bonds, sub = nqs.nqs_hypercube(N, 1)
    teacher = nqs.Model(N, w["M_teacher"], bonds, is_complex=True, prec=0)
    student = nqs.Model(N, M, bonds, is_complex=True, prec=w["prec"])
    pt = torch.from_numpy(synth.rbm_params(N, w["M_teacher"], True, sigma=0.1, seed=7)).to(dev)
    ps = torch.from_numpy(synth.rbm_params(N, M, True, sigma=0.01, seed=1234)).to(dev)
    ps = ps.to(student.param_dtype)
    idx = np.arange(2 ** N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N - 1, -1, -1)[None, :]) & 1
    states = torch.from_numpy((1 - 2 * bits).astype(np.int8)).to(dev)
    log_t = teacher.log_psi(pt, states)
    cdf = student.target_cdf(log_t)
    B = w["batch"]
    infos = []
    for k in range(warmup):
        sig, ltb, _ = student.target_draw(cdf, states, log_t, B, seed=1234, counter=k)
        infos.append(student.overlap_step(ps, sig, ltb, w["lr"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        sig, ltb, _ = student.target_draw(cdf, states, log_t, B, seed=1234,
                                          counter=warmup + k)
        infos.append(student.overlap_step(ps, sig, ltb, w["lr"]))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"workload": w["name"], "dtype": "f32", "ms_per_step": ms, "draws_per_step": B,
            "value": B / (ms * 1e-3), "unit": "samples/s", "steps_per_s": 1e3 / ms,
            "loss_first": infos[0]["loss"], "loss_last": infos[-1]["loss"],
            "training_set": 2 ** N}


def batch_instances(w):
    rng = np.random.default_rng(1234)
    Ns = rng.integers(w["Nmin"], w["Nmax"] + 1, size=w["K"])
    hs = rng.uniform(w["hmin"], w["hmax"], size=w["K"])
    return [int(x) for x in Ns], [float(x) for x in hs]


def bench_batch(nqs, synth, torch, name, steps, warmup):
    """The batched step (one persistent sampling launch for every chain of every ring,
    local energies in the sweep, stream-ordered SR of every ring) captured into one graph
    after one direct step, then replayed; the random stream advances on the device."""
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
    info = torch.zeros(w["K"] * nqs.SR_INFO_BYTES, dtype=torch.uint8, device=dev)
    counter = torch.zeros(1, dtype=torch.int64, device=dev)

    def step(discard):
        b.sample(params, chains, nch, S, discard, seed=1234, counter=0, samples=samples,
                 eloc=eloc, counter_dev=counter)
        b.sr_step_async(params, samples, eloc, ns, w["lr"], w["shift"], w["cg_tol"],
                        w["cg_maxiter"], workspace=ws, n_chains=nch, info=info)

    step(10)
    for _ in range(max(0, warmup - 1)):
        step(0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g, stream=s2):
            step(0)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = nqs.sr_infos_from_device(info, w["K"])
    ms_per_step = wall * 1e3 / steps
    # the sampling launch alone (tables + the persistent sweep with fused local energies)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    st = torch.cuda.current_stream()
    smp2 = torch.empty_like(samples)
    el2 = torch.empty_like(eloc)
    ch2 = chains.clone()
    reps = 5
    b2 = nqs.Batch(specs)   # its own job tables: the graph keeps the first handle's
    b2.sample(params, ch2, nch, S, 0, seed=77, counter=0, samples=smp2, eloc=el2)
    ev[0].record(st)
    for r in range(reps):
        b2.sample(params, ch2, nch, S, 0, seed=77, counter=(r + 1) * S, samples=smp2, eloc=el2)
    ev[1].record(st)
    torch.cuda.synchronize()
    samp_ms = ev[0].elapsed_time(ev[1]) / reps
    n_samp = C * S * w["K"]
    flops = float(sum(C * S * N * (w["alpha"] * N) * sweep_terms_flops(False) for N in Ns))
    ach = flops / (samp_ms * 1e-3)
    e_exact = [exact_tfim(N, h) for N, h in zip(Ns, hs)]
    de = [abs(i["energy_re"] - e) / abs(e) for i, e in zip(infos, e_exact)]
    return {
        "workload": name, "graph_replayed": True, "instances": w["K"],
        "n_sites_min": min(Ns), "n_sites_max": max(Ns), "chains_per_instance": C,
        "sweeps_per_step": S, "samples_per_step": n_samp, "cg_maxiter": w["cg_maxiter"],
        "ms_per_step": ms_per_step, "value": n_samp / (ms_per_step * 1e-3),
        "sr_iters_per_s": 1e3 / ms_per_step, "sampling_launch_ms": samp_ms,
        "cg_iters_max": max(i["cg_iters"] for i in infos),
        "converged_models": sum(i["converged"] for i in infos),
        "rel_energy_error_vs_exact_median": float(np.median(de)),
        "roofline": {"kernel": "k_sweep_batch (every chain of every ring, fused local energies)",
                     "bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": ach / PEAK_FP32_VALU, "traffic": None,
                     "algorithmic_flops": flops, "launch_ms": samp_ms},
    }


def exact_tfim(N, h, J=1.0):
    """Ferromagnetic periodic TFIM ring, free-fermion closed form (the exact energy each
    ring's VMC energy is compared with)."""
    k = (2 * np.arange(N) + 1) * np.pi / N
    return -float(np.sum(np.sqrt(J * J + h * h - 2 * J * h * np.cos(k))))


# ---- precision forms at a fixed energy error ------------------------------------------
def run_form(nqs, synth, torch, name, prec, iters):
    """SR trajectory of the workload in one precision form from the common start
    (parameters N(0, 0.01^2) from seed 1234, chains from seed 1234)."""
    s = Single(nqs, synth, torch, name, prec=prec)
    s.model.autotune(s.params, s.chains.repeat(s.S, 1), workspace=s.ws)
    energies, errs, walls = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(iters):
        info = s.step(max(10, s.S // 10) if k == 0 else 0)
        torch.cuda.synchronize()
        energies.append(info["energy_re"])
        errs.append(info["energy_err"])
        walls.append(time.perf_counter() - t0)
    return np.array(energies), np.array(errs), np.array(walls), s.S * s.C


def compare_forms(nqs, synth, torch, name, iters):
    """The same SR trajectory in the FP64, FP32 and BF16 forms. dE = |mean energy of the last
    10% of iterations - E_exact| / |E_exact|, sigma = error bar of that mean (the per-
    iteration error bars combined as independent). A low-precision form counts as reaching
    the FP64 form's accuracy when dE_form <= dE_fp64 + 2 sqrt(sigma_form^2 + sigma_fp64^2).
    time_to_dE: wall time until the 10-iteration running mean first reaches the largest final
    dE of the three forms (the error all of them reach)."""
    e_ref = golden(E_REF[name])
    out, runs = {}, {}
    for prec in (0, 1, 2):
        fname = FORM_NAMES[prec]
        log("forms: %s, %d SR iterations" % (fname, iters))
        runs[fname] = run_form(nqs, synth, torch, name, prec, iters)
    tail = max(1, iters // 10)
    for fname, (E, err, walls, n) in runs.items():
        steady = (walls[-1] - walls[0]) / max(1, len(walls) - 1)   # excludes the burn-in call
        mean = E[-tail:].mean()
        sig = np.sqrt(np.sum(err[-tail:] ** 2)) / tail / abs(e_ref)
        out[fname] = {"ms_per_iter": 1e3 * steady, "samples_per_s": n / steady,
                      "sr_iters_per_s": 1.0 / steady, "energy_final": float(mean),
                      "dE_final": float(abs(mean - e_ref) / abs(e_ref)), "sigma": float(sig)}
    ref = out["fp64"]
    for fname in ("fp32", "bf16"):
        o = out[fname]
        o["within_2sigma_of_fp64"] = bool(
            o["dE_final"] <= ref["dE_final"] + 2 * np.hypot(o["sigma"], ref["sigma"]))
        o["speedup_vs_fp64"] = ref["ms_per_iter"] / o["ms_per_iter"]
    target = max(v["dE_final"] for v in out.values())
    for fname, (E, err, walls, n) in runs.items():
        run_mean = np.array([E[max(0, k - 9):k + 1].mean() for k in range(len(E))])
        de = np.abs(run_mean - e_ref) / abs(e_ref)
        hit = np.nonzero(de <= target)[0]
        k = int(hit[0]) if hit.size else len(E) - 1
        out[fname]["iters_to_dE"] = k + 1
        out[fname]["time_to_dE_s"] = float(walls[k])
    return {"workload": name, "e_ref": e_ref, "e_ref_kind": "exact", "iters": iters,
            "tail_iters": tail, "dE_target": target, "forms": out}


# ---- the FP64 oracle on the host ----------------------------------------------------------
def cpu_baseline(name, seconds):
    """The FP64 oracle (plain numpy, unmodified: cached-angle Metropolis sweeps, local
    energies from log psi of every connected configuration, and the SR step with its dense S
    where that fits) on a bounded sample of the same workload."""
    import synth
    from oracle import hamiltonian as oh, lattice as ol, sampler as osamp, sr as osr
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        threads = 1
    w = WORKLOADS[name]
    N = w["L"] ** w["ndim"]
    M = w["alpha"] * N
    ob, osub = ol.hypercube(w["L"], w["ndim"], with_diagonals=w["diag"])
    om = oh.Model(N, M, ob, ham=w["ham"], J=w["J"], h=w["h"], marshall=w["marshall"],
                  sublattice=osub, move=w["move"], is_complex=w["cplx"])
    p = synth.rbm_params(N, M, w["cplx"], sigma=0.01, seed=1234)
    P = N + M + N * M
    with_sr = P <= 5000
    chains, sweeps = (64, 4) if N <= 64 else (16, 1)
    t0 = time.perf_counter()
    init = osamp.init_chains(om, chains, seed=1234)
    total = 0
    while True:
        smp, init, _ = osamp.sample_cached(om, p, init, sweeps, 0, seed=1234, counter=total)
        flat = smp.reshape(-1, N)
        el = oh.local_energy(om, p, flat)
        if with_sr:
            osr.sr_step(om, p, flat, el, w["lr"], w["shift"], w["cg_tol"], w["cg_maxiter"])
        total += flat.shape[0]
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    nproc, cpu = host_info()
    what = ("local energies and one SR step" if with_sr else
            "local energies (no SR: the oracle's dense S of %d parameters does not fit)" % P)
    return {"value": total / dt, "unit": "samples/s", "cores": int(threads), "kind": "oracle",
            "nproc": nproc, "cpu_model": cpu,
            "sample": "%s: %d chains x %d cached-angle sweeps per pass, %s per pass, %d passes "
                      "in %.1f s; cores = BLAS threads numpy used"
                      % (name, chains, sweeps, what, total // (chains * sweeps), dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=HEADLINE, choices=list(WORKLOADS))
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no other workloads, no form comparison)")
    ap.add_argument("--extra-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--forms-iters", type=int, default=500,
                    help="SR iterations per precision form in the FP64/FP32/BF16 comparison on "
                         "the 40-site ring (0 = skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--extra", default=None,
                    choices=(EXTRA_SINGLE + list(BATCH_WORKLOADS) +
                             [PT_WORKLOAD["name"], FF_WORKLOAD["name"], SUP_WORKLOAD["name"]]),
                    help="run only this one of the other workloads (--extra-steps steps) and "
                         "print its record (for profiling)")
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
    if args.extra:
        log("workload " + args.extra)
        if args.extra in BATCH_WORKLOADS:
            rec = bench_batch(nqs, synth, torch, args.extra, args.extra_steps, 2)
        elif args.extra == PT_WORKLOAD["name"]:
            rec = bench_pt(nqs, synth, torch, args.extra_steps, 2)
        elif args.extra == FF_WORKLOAD["name"]:
            rec = bench_ffnn(nqs, synth, torch, args.extra_steps, 2)
        elif args.extra == SUP_WORKLOAD["name"]:
            rec = bench_supervised(nqs, synth, torch, 5 * args.extra_steps, 3)
        else:
            s = Single(nqs, synth, torch, args.extra)
            rec = s.run(args.extra_steps, 2)
        print(json.dumps({"extra": args.extra, "record": rec}))
        return
    log("headline workload " + args.workload)
    head = Single(nqs, synth, torch, args.workload)
    r = head.run(args.steps, args.warmup)
    w = head.w
    log("headline: %.2f ms/step" % r["ms_per_step"])
    out = {
        "metric": METRIC, "value": r["value"], "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {0: "f64", 1: "f32", 2: "bf16"}[w["prec"]], "data": "synthetic",
        "config": {"workload": args.workload, "n_sites": head.N, "n_hidden": head.M,
                   "chains": head.C, "sweeps_per_step": head.S,
                   "samples_per_step": head.S * head.C, "cg_tol": w["cg_tol"],
                   "cg_maxiter": w["cg_maxiter"], "diag_shift": w["shift"], "lr": w["lr"]},
        "roofline": r["roofline"],
    }
    for k in ("sr_iters_per_s", "sampling_samples_per_s", "phase_ms", "kernel_ms",
              "cg_iters_mean", "real_move_fraction", "energy_last", "energy_err_last",
              "sv_tuning"):
        out[k] = r[k]
    if not args.no_extras:
        others = {}
        for name in EXTRA_SINGLE:
            if name == args.workload:
                continue
            log("workload " + name)
            s = Single(nqs, synth, torch, name)
            o = s.run(args.extra_steps, 2)
            o["dtype"] = {0: "f64", 1: "f32", 2: "bf16"}[s.prec]
            others[name] = o
            del s
        for name in BATCH_WORKLOADS:
            log("workload " + name + " (graph-replayed step)")
            others[name] = bench_batch(nqs, synth, torch, name, args.extra_steps, 2)
        log("workload " + PT_WORKLOAD["name"] + " (parallel tempering)")
        others[PT_WORKLOAD["name"]] = bench_pt(nqs, synth, torch, args.extra_steps, 2)
        log("workload " + FF_WORKLOAD["name"] + " (feed-forward network)")
        others[FF_WORKLOAD["name"]] = bench_ffnn(nqs, synth, torch, args.extra_steps, 2)
        log("workload " + SUP_WORKLOAD["name"] + " (supervised)")
        others[SUP_WORKLOAD["name"]] = bench_supervised(nqs, synth, torch, 5 * args.extra_steps, 3)
        out["other_workloads"] = others
        if args.forms_iters > 0:
            out["precision_forms"] = compare_forms(nqs, synth, torch,
                                                   "heisenberg1d_n40_cplx_fp32_alpha2",
                                                   args.forms_iters)
    if not args.no_cpu_baseline:
        log("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
