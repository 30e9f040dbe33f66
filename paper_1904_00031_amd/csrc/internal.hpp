// Host-side internals of libnqs: the model handle and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "common.hpp"

// arguments that fix the launches of a captured chunk of CG iterations
struct CgGraphKey {
  const void *ws = nullptr;
  const int8_t *sigma = nullptr;
  int64_t n = 0;
  double shift = 0, tol = 0;
  int maxiter = 0, sv_pairs = 0;
  bool operator==(const CgGraphKey &o) const {
    return ws == o.ws && sigma == o.sigma && n == o.n && shift == o.shift && tol == o.tol &&
           maxiter == o.maxiter && sv_pairs == o.sv_pairs;
  }
};

// the feed-forward network of a model (zero layers: an RBM). Offsets count elements of
// the value type (complex elements for complex models).
constexpr int kFfMaxLayers = 4;
constexpr int kFfMaxWidth = 512;
struct FfDev {
  int L, N, maxw;
  int w[kFfMaxLayers + 1];      // widths, w[0] = N
  int act[kFfMaxLayers];        // nqs_activation of each layer
  int64_t poff[kFfMaxLayers];   // b_l at poff[l], W_l [w[l+1]][w[l]] at poff[l] + w[l+1]
  int64_t toff[kFfMaxLayers];   // W_l transposed [w[l]][w[l+1]] at toff[l] of the table
  int zoff[kFfMaxLayers];       // columns of z_l (input of layer l, l >= 1) in a Z row
  int goff[kFfMaxLayers];       // columns of g_l = d log psi / d y_l in a G row
  int zcols, gcols;
  int64_t P, tab;               // parameters and table elements
};

struct nqs_model {
  int N, M, is_complex, prec, ham, move, marshall;
  // FFNN (ff.L > 0): the layer table d_fftab (W_l transposed, compute precision)
  FfDev ff = {};
  void *d_fftab = nullptr;
  // symmetric RBM: G site permutations (device [G][N]), alpha = M / G filters; the kernels
  // run the equivalent plain RBM on parameters expanded into d_pexp, with v_exp / g_exp
  // buffers for the Jacobian products (expanded layout, complex double)
  int G = 0, alpha = 0;
  int *d_perm = nullptr;
  void *d_pexp = nullptr;
  double *d_vexp = nullptr, *d_gexp = nullptr;
  int B[2], Btot;
  double J[2], h;
  int device;
  bool need_flip, need_bond;
  // device tables owned by the handle
  int *d_bonds = nullptr;          // [Btot][2]
  double *d_bond_diag = nullptr;   // [Btot]
  double *d_bond_off = nullptr;    // [Btot]
  void *d_tables = nullptr;        // parameter-derived tables (see Tables<T>)
  size_t tables_bytes = 0;
  void *tab_ptrs[14] = {};         // sub-buffers of d_tables, in Tables<T> member order
  int max_lds = 65536;             // dynamic LDS bytes a workgroup may use on this device
  int cu_count = 256;              // compute units of the device
  int sv_pairs = 2;                // plane-split S v: wavefront pairs per block (2 or 4)
  // grow-only scratch for nqs_log_psi_grad
  void *d_scratch = nullptr;
  size_t scratch_bytes = 0;
  // chunks of 8 CG iterations of nqs_sr_step replayed from a captured graph
  bool cg_graphs = true;
  hipStream_t cap_stream = nullptr;  // capture only (default priority)
  hipGraphExec_t cg_exec = nullptr;
  CgGraphKey cg_key;
  // solver-state copies read by the host while the next chunk runs: pinned host memory
  // (two slots) and the events that mark each copy complete
  void *cg_host = nullptr;
  hipEvent_t cg_ev[2] = {nullptr, nullptr};
  // timing of one kind of kernel launch (nqs_time_kernel): pairs of events recorded around
  // each kernel (or launcher) of it, summed by nqs_kernel_ms
  static constexpr int kTimeSlots = 8;
  int time_what = 0;
  mutable int time_n = 0;  // pairs recorded in the last timed call
  hipEvent_t time_ev[kTimeSlots][2] = {};
};

// timing marks: time_begin() when a timed call starts, then time_mark(0) / time_mark(1)
// around each of its kernels (events of the next pair)
inline void time_begin(const nqs_model *m, int what) {
  if (m->time_what == what) m->time_n = 0;
}
inline void time_mark(const nqs_model *m, int what, int which, hipStream_t st) {
  if (m->time_what != what || m->time_n >= nqs_model::kTimeSlots) return;
  const hipEvent_t e = m->time_ev[m->time_n][which];
  if (e) (void)hipEventRecord(e, st);
  if (which == 1) ++m->time_n;
}

// Device copy of a host-built job table. upload() copies only when the bytes differ from
// the previous upload, so a repeated call with the same buffers and sizes issues no
// host-to-device copy (and can then be captured into a graph).
struct JobBuffer {
  void *d = nullptr;
  size_t cap = 0;
  std::vector<char> last;
  hipError_t upload(const void *host, size_t bytes, hipStream_t st);
  void release();
};

// one model of a batch, with its buffers for one sampling call (device pointers)
struct BatchSampleItem {
  const nqs_model *m;
  const void *params;
  int8_t *chains;
  int n_chains;
  int8_t *samples;
  int64_t *n_acc;
  void *eloc;
  uint64_t seed;
};

struct nqs_batch {
  int K = 0;
  int is_complex = 0, prec = 0;
  std::vector<nqs_model *> models;
  JobBuffer tab_jobs, tab_map, sweep_jobs, sweep_map;   // sampling
  // SR step job tables, by slot. A fixed array: references to slots stay valid while
  // other slots are used (a growing container would move them).
  static constexpr int kSlots = 32;
  JobBuffer sr_bufs[kSlots];
  JobBuffer &buf(int slot) { return sr_bufs[slot < kSlots ? slot : kSlots - 1]; }
  // gathered solver states read by the host while the next chunk runs (pinned, two slots)
  void *cg_host = nullptr;
  size_t cg_host_bytes = 0;
  hipEvent_t cg_ev[2] = {nullptr, nullptr};
};

// one model of a batched Jacobian pass (device pointers into the model's workspace)
struct BatchGradItem {
  const nqs_model *m;
  int64_t n;
  const int8_t *sigma;
  void *Tm, *Vt, *vb;   // tanh rows, direction tables (compute precision)
  double *va;           // direction of a (complex double)
  double *ypart, *y, *ysum;  // JVP: per-chunk sums, O v, per-block sums of O v
  const double *u;      // VJP input
  void *part;           // VJP partial tiles
  double *out1, *out;   // VJP tile sums, packed result
  const int *skip;      // nonzero: the model's solve is finished, kernels return at once
};
// workspace pieces of one model in a batched Jacobian pass
struct BatchGradSizes {
  size_t Tm, Vt, vb, va, ypart, part, out1;
  int colsP;
  int64_t elems;
};
BatchGradSizes batch_grad_sizes(const nqs_model *m, int64_t n);
// slot: first of the batch's job-table slots the call may use (theta/tanh 2, JVP 3, VJP 4)
hipError_t launch_theta_tanh_batch(nqs_batch *b, const std::vector<BatchGradItem> &items,
                                   int slot, hipStream_t st);
hipError_t launch_jvp_batch(nqs_batch *b, const std::vector<BatchGradItem> &items, int slot,
                            hipStream_t st);
hipError_t launch_vjp_batch(nqs_batch *b, const std::vector<BatchGradItem> &items,
                            bool to_params, int slot, hipStream_t st);
hipError_t launch_tables_batch(nqs_batch *b, const std::vector<const void *> &params,
                               hipStream_t st);

// tables of every model, then every chain of every model in one persistent launch; the
// sweep base is counter, or *counter_dev (advanced by n_discard + n_sweeps afterwards)
hipError_t launch_sample_batch(nqs_batch *b, const std::vector<BatchSampleItem> &items,
                               int n_sweeps, int n_discard, uint64_t counter,
                               uint64_t *counter_dev, hipStream_t st);

// compute precision of the VALU kernels: double for NQS_F64, float otherwise
inline bool use_double(const nqs_model *m) { return m->prec == NQS_F64; }

// ---- symmetric RBM (symm.hip) -------------------------------------------------------
inline int64_t n_params_exp(const nqs_model *m) {
  return int64_t(m->N) + m->M + int64_t(m->N) * m->M;
}
inline int64_t n_params_model(const nqs_model *m) {
  if (m->ff.L) return m->ff.P;
  return m->G ? 1 + m->alpha + int64_t(m->alpha) * m->N : n_params_exp(m);
}
// p_exp (expanded RBM, master precision) from p_sym: a_i = a, b_fG+g = b_f,
// W_fG+g,perm[g][i] = W_fi
hipError_t launch_symm_expand(const nqs_model *m, const void *p_sym, void *p_exp, hipStream_t st);
// the same expansion of a direction in (complex) double; skip (may be NULL): nonzero -> return
hipError_t launch_symm_expand_dir(const nqs_model *m, const double *v_sym, double *v_exp,
                                  const int *skip, hipStream_t st);
// g_sym = E^T g_exp (sum over the symmetry copies of every parameter), (complex) double
hipError_t launch_symm_reduce(const nqs_model *m, const double *g_exp, double *g_sym,
                              hipStream_t st);
// the parameters the kernels read: p itself, or its expansion into d_pexp (launched here)
const void *model_params(nqs_model *m, const void *p, hipStream_t st, hipError_t *err);

DevModel dev_model(const nqs_model *m);

// ---- launchers (return hipError_t of the launch) -----------------------------------
hipError_t launch_tables(const nqs_model *m, const void *params, hipStream_t st);
hipError_t launch_chain_init(const nqs_model *m, int8_t *sig, int n_chains, uint64_t seed,
                             int chain_offset, hipStream_t st);
// parallel tempering of nqs_sample_pt: n_rep replicas per chain (chain_sigma [C R][N]),
// temperature index of every replica (device [C R], in/out), accepted exchanges per chain
struct PtArgs {
  int n_rep;
  int *temp;
  int64_t *n_swap;
};
// whether the sweep kernels temper this model (not the wide float sweep)
inline bool pt_supported(const nqs_model *m) { return use_double(m) || m->M <= 256; }

// scratch: device memory of sweep_scratch_bytes(m, n_chains) bytes for the chains' angles
// of the wide sweep (NULL: the sweep forms them itself). pt: tempering (n_chains then
// counts replicas, C R), or NULL
hipError_t launch_sweep(const nqs_model *m, int8_t *chain_sigma, int n_chains, int n_sweeps,
                        int n_discard, uint64_t seed, uint64_t counter, int chain_offset,
                        int8_t *samples, int64_t *n_acc, void *eloc, void *scratch,
                        hipStream_t st, const PtArgs *pt = nullptr);
size_t sweep_scratch_bytes(const nqs_model *m, int n_chains);
// local energies from rows Tm [n][M] of tanh(theta) (compute precision)
hipError_t launch_local_energy(const nqs_model *m, const int8_t *sigma, const void *Tm,
                               int64_t n, void *eloc, hipStream_t st);
hipError_t launch_log_psi(const nqs_model *m, const int8_t *sigma, int64_t n, void *out,
                          hipStream_t st);

// ---- Jacobian products (grad.hip) ---------------------------------------------------
// scratch layout for one JVP / VJP pair, sized by grad_scratch_bytes
struct GradPlan {
  int Jtiles;    // 16-row tiles over hidden rows 0..M of the VJP output
  int Itiles;    // 16-column tiles over site columns 0..N of the VJP output
  int JT, NT;    // tiles per wavefront (hidden x site) in the VJP
  int splits;    // sample splits of the VJP (grid y)
  int64_t per_split;  // samples per split (multiple of 16)
  int groups;    // first-level reduction groups of the VJP partials
  bool fused;    // all VJP tiles fit one block: S v in one pass (k_sv)
  bool wide;     // FP32 VJP with every site tile in one block (k_vjp_wide, spin quads)
  bool pair;     // fused, complex FP32 and N <= 63: plane-split pairs on spin masks (k_svc)
  bool tbf;      // BF16 form: T rows of the Jacobian products stored as bfloat16
  int pairs;     // wavefront pairs per k_svc block
  int jchunks;   // hidden chunks (8 tiles FP32, 4 FP64) of the JVP / tanh kernels (grid y)
  int64_t jvp_blocks; // sample tiles of 64 in the JVP / tanh kernels
};
GradPlan grad_plan(const nqs_model *m, int64_t n);
size_t grad_scratch_bytes(const nqs_model *m, int64_t n);

// v (double, params layout) -> direction tables in compute precision, in scratch
// split: also write the bf16 split of the direction (read only by the separate JVP kernel)
hipError_t launch_prep_dir(const nqs_model *m, const void *v, void *scratch, bool split,
                           hipStream_t st);
// T = tanh(theta) of every sample into scratch (needed by launch_jvp / launch_vjp_partials
// and the local energies from rows); for_grad: rows for the Jacobian contractions, which
// the BF16 form rounds to bfloat16
hipError_t launch_theta_tanh(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                             bool for_grad, hipStream_t st);
// y[s] = (O v)[s] with the direction prepared by launch_prep_dir; ysum (may be NULL)
// receives per-block partial sums of y (complex double) for the centering
hipError_t launch_jvp(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                      double *y, double *ysum_part, const int *skip, hipStream_t st);
// raw partials of O^dagger u into scratch (u: complex/real double [n])
hipError_t launch_vjp_partials(const nqs_model *m, const int8_t *sigma, int64_t n,
                               const double *u, void *scratch, const int *skip,
                               hipStream_t st, bool reduce = true);
// fused S v (requires plan.fused): partials of O^dagger y with y = O v, plus per-block sums
// of y (complex double, plan.splits entries), then the first reduction level
hipError_t launch_sv(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                     double *ysum_part, const int *skip, hipStream_t st, bool reduce = true);
struct GradBuffers {
  void *Tm;        // tanh(theta) rows [n][M] (compute precision)
  void *Vt, *vb;   // direction tables in compute precision
  double *va;      // visible part of the direction, complex double
  double *out1;    // first-level VJP sums [groups][Jtiles*16*Itiles*16] complex double
  void *part;      // per-split VJP partial tiles [splits][Jtiles*16][Itiles*16], compute precision
};
GradBuffers grad_buffers(const nqs_model *m, int64_t n, void *scratch);
// out[k] = sum of partials (double, params layout)
hipError_t launch_vjp_reduce(const nqs_model *m, int64_t n, void *scratch, double *out,
                             const int *skip, hipStream_t st);

// ---- feed-forward network (ffnn.hip) ----------------------------------------------------
// every launcher refreshes nothing: launch_ff_tables(params) first
hipError_t launch_ff_tables(const nqs_model *m, const void *params, hipStream_t st);
hipError_t launch_ff_log_psi(const nqs_model *m, const void *params, const int8_t *sigma,
                             int64_t n, void *out, hipStream_t st);
hipError_t launch_ff_local_energy(const nqs_model *m, const void *params, const int8_t *sigma,
                                  int64_t n, void *eloc, hipStream_t st);
hipError_t launch_ff_sweep(const nqs_model *m, const void *params, int8_t *chain_sigma,
                           int n_chains, int n_sweeps, int n_discard, uint64_t seed,
                           uint64_t counter, int chain_offset, int8_t *samples, int64_t *n_acc,
                           hipStream_t st);
// scratch of the Jacobian products of n samples: Z and G rows, direction tables, VJP partials
size_t ff_grad_scratch_bytes(const nqs_model *m, int64_t n);
// forward and backward pass of every sample: Z (layer inputs) and G rows into scratch
hipError_t launch_ff_fb(const nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                        void *scratch, hipStream_t st);
// y = O v (complex double [n]) and per-block partial sums of y (ysum may be NULL); v:
// (complex) double, params layout; skip (may be NULL): nonzero -> kernels return
hipError_t launch_ff_jvp(const nqs_model *m, const void *params, const int8_t *sigma,
                         int64_t n, const double *v, void *scratch, double *y, double *ysum,
                         const int *skip, hipStream_t st);
int64_t ff_jvp_blocks(const nqs_model *m, int64_t n);
// out = O^dagger u ((complex) double, params layout)
hipError_t launch_ff_vjp(const nqs_model *m, const int8_t *sigma, int64_t n, const double *u,
                         void *scratch, double *out, const int *skip, hipStream_t st);

// ---- supervised learning (overlap.hip) -------------------------------------------------
hipError_t launch_target_cdf(const nqs_model *m, const void *log_t, int64_t n_states,
                             double *cdf, hipStream_t st);
hipError_t launch_target_draw(const nqs_model *m, const double *cdf, int64_t n_states,
                              const int8_t *states, const void *log_t, int64_t n,
                              uint64_t seed, uint64_t counter, int8_t *sigma, void *log_t_out,
                              int64_t *index, hipStream_t st);
size_t overlap_scratch_bytes(const nqs_model *m, int64_t n);
nqs_status overlap_step_impl(nqs_model *m, void *params, const int8_t *sigma,
                             const void *log_t, int64_t n, double lr, void *scratch,
                             nqs_overlap_info *info, hipStream_t st);

// ---- SR (sr.hip) --------------------------------------------------------------------
size_t sr_workspace_bytes(const nqs_model *m, int64_t n);
nqs_status sr_prepare_impl(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                           void *ws, size_t ws_bytes, hipStream_t st);
nqs_status sr_matvec_impl(nqs_model *m, const int8_t *sigma, int64_t n, void *ws,
                          size_t ws_bytes, const void *v, double lambda, void *out,
                          hipStream_t st);
nqs_status autotune_impl(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                         void *ws, size_t ws_bytes, nqs_tune_report *rep, hipStream_t st);
// async: stream-ordered (info is a device pointer); otherwise synchronising (host info)
nqs_status sr_step_impl(nqs_model *m, void *params, const int8_t *sigma, const void *eloc,
                        int64_t n, int64_t n_chains, double lr, double diag_shift, double cg_tol,
                        int cg_maxiter, void *ws, size_t ws_bytes, nqs_sr_info *info, bool async,
                        hipStream_t st);

size_t batch_sr_workspace_bytes(nqs_batch *b, const int64_t *n_samples);
nqs_status batch_sr_step_impl(nqs_batch *b, void *params, const int8_t *samples,
                              const void *eloc, const int64_t *n_samples, const int32_t *n_chains,
                              double lr, double diag_shift, double cg_tol, int cg_maxiter,
                              void *ws, size_t ws_bytes, nqs_sr_info *info, bool async,
                              hipStream_t st);
