// Batches of independent models (uneven lattice sizes, couplings and hidden-unit counts)
// advanced together: one launch builds every model's tables and one persistent launch
// runs every chain of every model (Sec. 2.2.5 Metropolis sampling with local energies).
// Buffers of the models are concatenated in model order; job tables that map each block
// to its model are built on the host and uploaded only when they change.
#include <string.h>

#include <cmath>

#include <new>
#include <vector>

#include "internal.hpp"

namespace {

inline nqs_status dev(hipError_t e) { return e == hipSuccess ? NQS_OK : NQS_EDEVICE; }

inline int64_t n_params_of(const nqs_model *m) {
  return int64_t(m->N) + m->M + int64_t(m->N) * m->M;
}

// bytes of one parameter in the master precision, and of one per-sample result
inline size_t param_bytes(const nqs_model *m) {
  return (m->prec == NQS_F64 ? 8 : 4) * (m->is_complex ? 2 : 1);
}
inline size_t value_bytes(const nqs_model *m) { return m->is_complex ? 16 : 8; }

}  // namespace

hipError_t JobBuffer::upload(const void *host, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (d && last.size() == bytes && memcmp(last.data(), host, bytes) == 0) return hipSuccess;
  // queued work may still read the previous table
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (bytes > cap) {
    if (d) (void)hipFree(d);
    d = nullptr;
    cap = 0;
    if ((e = hipMalloc(&d, bytes)) != hipSuccess) return e;
    cap = bytes;
  }
  if ((e = hipMemcpy(d, host, bytes, hipMemcpyHostToDevice)) != hipSuccess) return e;
  last.assign((const char *)host, (const char *)host + bytes);
  return hipSuccess;
}

void JobBuffer::release() {
  if (d) (void)hipFree(d);
  d = nullptr;
  cap = 0;
  last.clear();
}

extern "C" {

nqs_status nqs_batch_create(const nqs_model_desc *descs, int32_t n_models, nqs_batch **out) {
  if (!descs || !out || n_models < 1) return NQS_EINVAL;
  *out = nullptr;
  for (int k = 0; k < n_models; ++k)
    if (descs[k].is_complex != descs[0].is_complex || descs[k].prec != descs[0].prec ||
        descs[k].n_symm != 0 || descs[k].n_layers != 0)
      return NQS_EINVAL;
  nqs_batch *b = new (std::nothrow) nqs_batch();
  if (!b) return NQS_ENOMEM;
  b->K = n_models;
  b->is_complex = descs[0].is_complex ? 1 : 0;
  b->prec = descs[0].prec;
  for (int k = 0; k < n_models; ++k) {
    nqs_model *m = nullptr;
    nqs_status s = nqs_model_create(&descs[k], &m);
    if (s != NQS_OK) {
      nqs_batch_destroy(b);
      return s;
    }
    b->models.push_back(m);
  }
  *out = b;
  return NQS_OK;
}

void nqs_batch_destroy(nqs_batch *b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  for (nqs_model *m : b->models) nqs_model_destroy(m);
  b->tab_jobs.release();
  b->tab_map.release();
  b->sweep_jobs.release();
  b->sweep_map.release();
  for (JobBuffer &j : b->sr_bufs) j.release();
  if (b->cg_host) (void)hipHostFree(b->cg_host);
  for (hipEvent_t e : b->cg_ev)
    if (e) (void)hipEventDestroy(e);
  delete b;
}

int64_t nqs_batch_n_params(const nqs_batch *b, int32_t k) {
  if (!b || k < 0 || k >= b->K) return -1;
  return n_params_of(b->models[k]);
}

nqs_status nqs_batch_chain_init(nqs_batch *b, int8_t *chain_sigma, const int32_t *n_chains,
                                uint64_t seed, void *stream) {
  if (!b || !chain_sigma || !n_chains) return NQS_EINVAL;
  for (int k = 0; k < b->K; ++k)
    if (n_chains[k] < 1) return NQS_EINVAL;
  size_t off = 0;
  for (int k = 0; k < b->K; ++k) {
    const nqs_model *m = b->models[k];
    hipError_t e = launch_chain_init(m, chain_sigma + off, n_chains[k], seed ^ uint64_t(k), 0,
                                     (hipStream_t)stream);
    if (e != hipSuccess) return NQS_EDEVICE;
    off += size_t(n_chains[k]) * m->N;
  }
  return NQS_OK;
}

nqs_status nqs_batch_sample(nqs_batch *b, const void *params, int8_t *chain_sigma,
                            const int32_t *n_chains, int32_t n_sweeps, int32_t n_discard,
                            uint64_t seed, uint64_t counter, uint64_t *counter_dev,
                            int8_t *samples, int64_t *n_accepted, void *eloc, void *stream) {
  if (!b || !params || !chain_sigma || !n_chains || !samples || n_sweeps < 1 || n_discard < 0)
    return NQS_EINVAL;
  for (int k = 0; k < b->K; ++k)
    if (n_chains[k] < 1) return NQS_EINVAL;
  std::vector<BatchSampleItem> items;
  size_t op = 0, oc = 0, os = 0, oe = 0, oa = 0;
  for (int k = 0; k < b->K; ++k) {
    const nqs_model *m = b->models[k];
    BatchSampleItem it;
    it.m = m;
    it.params = (const char *)params + op;
    it.chains = chain_sigma + oc;
    it.n_chains = n_chains[k];
    it.samples = samples + os;
    it.n_acc = n_accepted ? n_accepted + oa : nullptr;
    it.eloc = eloc ? (void *)((char *)eloc + oe) : nullptr;
    it.seed = seed ^ uint64_t(k);
    items.push_back(it);
    op += size_t(n_params_of(m)) * param_bytes(m);
    oc += size_t(n_chains[k]) * m->N;
    os += size_t(n_sweeps) * n_chains[k] * m->N;
    oe += size_t(n_sweeps) * n_chains[k] * value_bytes(m);
    oa += size_t(n_chains[k]);
  }
  return dev(launch_sample_batch(b, items, n_sweeps, n_discard, counter, counter_dev,
                                 (hipStream_t)stream));
}

size_t nqs_batch_sr_workspace_bytes(nqs_batch *b, const int64_t *n_samples) {
  if (!b || !n_samples) return 0;
  for (int k = 0; k < b->K; ++k)
    if (n_samples[k] < 2) return 0;
  return batch_sr_workspace_bytes(b, n_samples);
}

static nqs_status batch_sr_checked(nqs_batch *b, void *params, const int8_t *samples,
                                   const void *eloc, const int64_t *n_samples,
                                   const int32_t *n_chains, double lr, double diag_shift,
                                   double cg_tol, int32_t cg_maxiter, void *workspace,
                                   size_t ws_bytes, nqs_sr_info *info, bool async, void *stream) {
  if (!b || !params || !samples || !eloc || !n_samples || !workspace || cg_maxiter < 1 ||
      !(diag_shift >= 0) || !(cg_tol >= 0) || !std::isfinite(lr) || (async && !info))
    return NQS_EINVAL;
  for (int k = 0; k < b->K; ++k) {
    if (n_samples[k] < 2) return NQS_EINVAL;
    if (n_chains && (n_chains[k] < 0 || n_chains[k] == 1 || n_chains[k] > n_samples[k] ||
                     (n_chains[k] > 0 && n_samples[k] % n_chains[k])))
      return NQS_EINVAL;
  }
  return batch_sr_step_impl(b, params, samples, eloc, n_samples, n_chains, lr, diag_shift, cg_tol,
                            cg_maxiter, workspace, ws_bytes, info, async, (hipStream_t)stream);
}

nqs_status nqs_batch_sr_step(nqs_batch *b, void *params, const int8_t *samples,
                             const void *eloc, const int64_t *n_samples, const int32_t *n_chains,
                             double lr, double diag_shift, double cg_tol, int32_t cg_maxiter,
                             void *workspace, size_t ws_bytes, nqs_sr_info *info, void *stream) {
  return batch_sr_checked(b, params, samples, eloc, n_samples, n_chains, lr, diag_shift, cg_tol,
                          cg_maxiter, workspace, ws_bytes, info, false, stream);
}

nqs_status nqs_batch_sr_step_async(nqs_batch *b, void *params, const int8_t *samples,
                                   const void *eloc, const int64_t *n_samples,
                                   const int32_t *n_chains, double lr, double diag_shift,
                                   double cg_tol, int32_t cg_maxiter, void *workspace,
                                   size_t ws_bytes, nqs_sr_info *info, void *stream) {
  return batch_sr_checked(b, params, samples, eloc, n_samples, n_chains, lr, diag_shift, cg_tol,
                          cg_maxiter, workspace, ws_bytes, info, true, stream);
}

}  // extern "C"
