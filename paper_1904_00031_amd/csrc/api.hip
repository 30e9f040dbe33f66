// C ABI of libnqs: argument validation, model handles and dispatch to the kernels.
#include <limits.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "internal.hpp"

// Scratch of nqs_log_psi_grad_noalloc: one fixed array per device, held for the life of
// the process. Host code never passes this name to a kernel (on the host it is only a
// stand-in for the symbol); it uses the device address returned by hipGetSymbolAddress,
// looked up once per device with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (resolved on the first call there)
nqs_status noalloc_scratch(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NQS_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return NQS_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NQS_OK;
}

__global__ void k_zero(int64_t count, double *x) {
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < count;
       k += int64_t(gridDim.x) * blockDim.x)
    x[k] = 0.0;
}

inline unsigned grid_for(int64_t count) {
  int64_t b = (count + 255) / 256;
  return unsigned(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

nqs_status dev(hipError_t e) { return e == hipSuccess ? NQS_OK : NQS_EDEVICE; }

int64_t n_params_of(const nqs_model *m) { return n_params_model(m); }

nqs_status ensure_scratch(nqs_model *m, size_t bytes) {
  if (m->scratch_bytes >= bytes) return NQS_OK;
  if (m->d_scratch) {
    if (hipDeviceSynchronize() != hipSuccess) return NQS_EDEVICE;
    (void)hipFree(m->d_scratch);
    m->d_scratch = nullptr;
    m->scratch_bytes = 0;
  }
  if (hipMalloc(&m->d_scratch, bytes) != hipSuccess) return NQS_ENOMEM;
  m->scratch_bytes = bytes;
  return NQS_OK;
}

}  // namespace

DevModel dev_model(const nqs_model *m) {
  // zero-filled: copies of it go into job tables that are compared byte by byte
  DevModel d;
  memset(static_cast<void *>(&d), 0, sizeof d);
  d.N = m->N;
  d.M = m->M;
  d.B0 = m->B[0];
  d.Btot = m->Btot;
  d.ham = m->ham;
  d.move = m->move;
  d.h = m->h;
  d.bonds = m->d_bonds;
  d.bond_diag = m->d_bond_diag;
  d.bond_off = m->d_bond_off;
  return d;
}

extern "C" {

const char *nqs_status_string(nqs_status s) {
  switch (s) {
    case NQS_OK: return "ok";
    case NQS_ENOTCONV: return "conjugate gradients reached cg_maxiter before cg_tol";
    case NQS_EINVAL: return "invalid argument";
    case NQS_ENOMEM: return "out of device memory or workspace too small";
    case NQS_EDEVICE: return "HIP runtime or launch error";
    case NQS_ENONFINITE: return "non-finite energy, force or CG scalar";
    case NQS_EUNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

nqs_status nqs_hypercube(int32_t L, int32_t ndim, int32_t with_diagonals, int32_t *bonds0,
                         int32_t *bonds1, int8_t *sublattice, int32_t *n_bonds) {
  if (L < 3 || L > 1024 || (ndim != 1 && ndim != 2) || !bonds0 || !sublattice || !n_bonds)
    return NQS_EINVAL;
  if (with_diagonals && (ndim != 2 || !bonds1)) return NQS_EINVAL;
  const int n = ndim == 1 ? L : L * L;
  int b0 = 0, b1 = 0;
  for (int s = 0; s < n; ++s) {
    const int x = s % L, y = ndim == 2 ? s / L : 0;
    sublattice[s] = int8_t((x + y) % 2);
    // +e_x
    bonds0[2 * b0] = s;
    bonds0[2 * b0 + 1] = (x + 1) % L + L * y;
    ++b0;
    if (ndim == 2) {
      bonds0[2 * b0] = s;
      bonds0[2 * b0 + 1] = x + L * ((y + 1) % L);
      ++b0;
      if (with_diagonals) {
        bonds1[2 * b1] = s;
        bonds1[2 * b1 + 1] = (x + 1) % L + L * ((y + 1) % L);
        ++b1;
        bonds1[2 * b1] = s;
        bonds1[2 * b1 + 1] = (x + 1) % L + L * ((y + L - 1) % L);
        ++b1;
      }
    }
  }
  n_bonds[0] = b0;
  n_bonds[1] = b1;
  return NQS_OK;
}

nqs_status nqs_hypercube_translations(int32_t L, int32_t ndim, int32_t *perm) {
  if (L < 3 || (ndim != 1 && ndim != 2) || !perm) return NQS_EINVAL;
  const int n = ndim == 1 ? L : L * L;
  if (n > 1024) return NQS_EINVAL;
  for (int g = 0; g < n; ++g) {
    const int gx = g % L, gy = ndim == 2 ? g / L : 0;
    for (int s = 0; s < n; ++s) {
      const int x = s % L, y = ndim == 2 ? s / L : 0;
      perm[int64_t(g) * n + s] = (x + gx) % L + (ndim == 2 ? L * ((y + gy) % L) : 0);
    }
  }
  return NQS_OK;
}

nqs_status nqs_model_create(const nqs_model_desc *d, nqs_model **out) {
  if (!d || !out) return NQS_EINVAL;
  *out = nullptr;
  if (d->n_sites < 2 || d->n_sites > 1024 || d->n_hidden < 1 || d->n_hidden > 2048)
    return NQS_EINVAL;
  if (d->prec < NQS_F64 || d->prec > NQS_BF16) return NQS_EINVAL;
  if (d->ham != NQS_TFIM && d->ham != NQS_HEISENBERG) return NQS_EINVAL;
  if (d->move != NQS_MOVE_FLIP && d->move != NQS_MOVE_EXCHANGE) return NQS_EINVAL;
  if (!isfinite(d->J[0]) || !isfinite(d->J[1]) || !isfinite(d->h)) return NQS_EINVAL;
  for (int c = 0; c < 2; ++c) {
    if (d->n_bonds[c] < 0 || d->n_bonds[c] > 8 * d->n_sites) return NQS_EINVAL;
    if (d->n_bonds[c] > 0 && !d->bonds[c]) return NQS_EINVAL;
    for (int b = 0; b < d->n_bonds[c]; ++b) {
      int i = d->bonds[c][2 * b], k = d->bonds[c][2 * b + 1];
      if (i < 0 || k < 0 || i >= d->n_sites || k >= d->n_sites || i == k) return NQS_EINVAL;
    }
  }
  if (d->move == NQS_MOVE_EXCHANGE && (d->n_bonds[0] < 1 || d->n_sites % 2)) return NQS_EINVAL;
  if (d->marshall && !d->sublattice) return NQS_EINVAL;
  if (d->n_symm < 0 || (d->n_symm > 0 && (!d->symm || d->n_hidden % d->n_symm))) return NQS_EINVAL;
  if (d->n_layers < 0 || d->n_layers > kFfMaxLayers) return NQS_EINVAL;
  if (d->n_layers > 0) {
    if (!d->layer_sizes || !d->activations || d->n_symm > 0) return NQS_EINVAL;
    for (int l = 0; l < d->n_layers; ++l)
      if (d->layer_sizes[l] < 1 || d->layer_sizes[l] > kFfMaxWidth ||
          (d->activations[l] != NQS_ACT_LNCOSH && d->activations[l] != NQS_ACT_TANH))
        return NQS_EINVAL;
    if (d->prec == NQS_BF16) return NQS_EUNSUPPORTED;
  }
  if (d->n_symm > 0) {
    std::vector<char> seen(d->n_sites);
    for (int g = 0; g < d->n_symm; ++g) {
      std::fill(seen.begin(), seen.end(), 0);
      for (int i = 0; i < d->n_sites; ++i) {
        const int k = d->symm[int64_t(g) * d->n_sites + i];
        if (k < 0 || k >= d->n_sites || seen[k]) return NQS_EINVAL;
        seen[k] = 1;
      }
    }
  }

  nqs_model *m = new (std::nothrow) nqs_model();
  if (!m) return NQS_ENOMEM;
  m->N = d->n_sites;
  m->M = d->n_layers > 0 ? d->layer_sizes[0] : d->n_hidden;
  if (d->n_layers > 0) {
    // the network's layout: parameter, table, Z-row and G-row offsets of every layer
    FfDev &f = m->ff;
    f.L = d->n_layers;
    f.N = d->n_sites;
    f.w[0] = d->n_sites;
    f.maxw = d->n_sites;
    int64_t p = 0, t = 0;
    int zc = 0, gc = 0;
    for (int l = 0; l < f.L; ++l) {
      f.w[l + 1] = d->layer_sizes[l];
      f.act[l] = d->activations[l];
      f.maxw = f.w[l + 1] > f.maxw ? f.w[l + 1] : f.maxw;
      f.poff[l] = p;
      p += int64_t(f.w[l + 1]) * (1 + f.w[l]);
      f.toff[l] = t;
      t += int64_t(f.w[l]) * f.w[l + 1];
      f.goff[l] = gc;
      gc += f.w[l + 1];
      f.zoff[l] = l == 0 ? 0 : zc;
      if (l > 0) zc += f.w[l];
    }
    f.P = p;
    f.tab = t;
    f.zcols = zc;
    f.gcols = gc;
  }
  m->is_complex = d->is_complex ? 1 : 0;
  m->prec = d->prec;
  m->ham = d->ham;
  m->move = d->move;
  m->marshall = d->marshall ? 1 : 0;
  m->B[0] = d->n_bonds[0];
  m->B[1] = d->n_bonds[1];
  m->Btot = m->B[0] + m->B[1];
  m->J[0] = d->J[0];
  m->J[1] = d->J[1];
  m->h = d->h;
  m->need_flip = m->move == NQS_MOVE_FLIP || m->ham == NQS_TFIM;
  m->need_bond = m->move == NQS_MOVE_EXCHANGE || m->ham == NQS_HEISENBERG;
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return NQS_EDEVICE;
  }
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device) ==
            hipSuccess &&
        lds > 0)
      m->max_lds = lds;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) ==
            hipSuccess &&
        cus > 0)
      m->cu_count = cus;
  }

  // bond lists with their diagonal and exchange coefficients
  std::vector<int> bonds(2 * size_t(m->Btot > 0 ? m->Btot : 1));
  std::vector<double> diag(m->Btot > 0 ? m->Btot : 1), off(m->Btot > 0 ? m->Btot : 1);
  int q = 0;
  for (int c = 0; c < 2; ++c) {
    for (int b = 0; b < m->B[c]; ++b, ++q) {
      const int i = d->bonds[c][2 * b], k = d->bonds[c][2 * b + 1];
      bonds[2 * q] = i;
      bonds[2 * q + 1] = k;
      if (m->ham == NQS_TFIM) {
        diag[q] = -m->J[c];
        off[q] = 0.0;
      } else {
        double sgn = (m->marshall && d->sublattice[i] != d->sublattice[k]) ? -1.0 : 1.0;
        diag[q] = m->J[c];
        off[q] = 2.0 * m->J[c] * sgn;
      }
    }
  }
  const size_t nb = size_t(m->Btot > 0 ? m->Btot : 1);
  bool ok = hipMalloc(&m->d_bonds, 2 * nb * sizeof(int)) == hipSuccess &&
            hipMalloc(&m->d_bond_diag, nb * sizeof(double)) == hipSuccess &&
            hipMalloc(&m->d_bond_off, nb * sizeof(double)) == hipSuccess;
  if (ok)
    ok = hipMemcpy(m->d_bonds, bonds.data(), 2 * nb * sizeof(int), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(m->d_bond_diag, diag.data(), nb * sizeof(double), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(m->d_bond_off, off.data(), nb * sizeof(double), hipMemcpyHostToDevice) ==
             hipSuccess;

  // parameter-derived tables, in Tables<T> member order
  const size_t es = (use_double(m) ? 8 : 4) * (m->is_complex ? 2 : 1);
  const size_t NM = size_t(m->N) * m->M, BM = size_t(m->Btot) * m->M;
  size_t sizes[14] = {NM * es,
                      size_t(m->M) * es,
                      m->need_flip ? NM * es : 0,
                      m->need_flip ? NM * es : 0,
                      m->need_bond ? BM * es : 0,
                      m->need_bond ? BM * es : 0,
                      0,
                      0,
                      0,
                      0,
                      size_t(m->N) * 32,
                      nb * 32,
                      size_t(m->N) * 16,
                      m->move == NQS_MOVE_EXCHANGE ? size_t(m->B[0]) * m->M * es : 0};
  size_t offs[14], total = 0;
  for (int k = 0; k < 14; ++k) {
    offs[k] = total;
    total += (sizes[k] + 255) / 256 * 256;
  }
  if (ok) ok = hipMalloc(&m->d_tables, total) == hipSuccess;
  // symmetric RBM: the permutations and the expanded-parameter buffers
  if (ok && d->n_symm > 0) {
    m->G = d->n_symm;
    m->alpha = m->M / m->G;
    const size_t pe = size_t(n_params_exp(m)) * (m->is_complex ? 2 : 1);
    ok = hipMalloc(&m->d_perm, size_t(m->G) * m->N * sizeof(int)) == hipSuccess &&
         hipMalloc(&m->d_pexp, pe * (use_double(m) ? 8 : 4)) == hipSuccess &&
         hipMalloc(&m->d_vexp, pe * 8) == hipSuccess &&
         hipMalloc(&m->d_gexp, pe * 8) == hipSuccess;
    if (ok)
      ok = hipMemcpy(m->d_perm, d->symm, size_t(m->G) * m->N * sizeof(int),
                     hipMemcpyHostToDevice) == hipSuccess;
  }
  if (ok && m->ff.L)
    ok = hipMalloc(&m->d_fftab, size_t(m->ff.tab) * es) == hipSuccess;
  if (!ok) {
    nqs_model_destroy(m);
    return NQS_ENOMEM;
  }
  m->tables_bytes = total;
  for (int k = 0; k < 14; ++k) m->tab_ptrs[k] = sizes[k] ? (char *)m->d_tables + offs[k] : nullptr;
  *out = m;
  return NQS_OK;
}

void nqs_model_destroy(nqs_model *m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  if (m->d_bonds) (void)hipFree(m->d_bonds);
  if (m->d_bond_diag) (void)hipFree(m->d_bond_diag);
  if (m->d_bond_off) (void)hipFree(m->d_bond_off);
  if (m->d_tables) (void)hipFree(m->d_tables);
  if (m->d_fftab) (void)hipFree(m->d_fftab);
  if (m->d_perm) (void)hipFree(m->d_perm);
  if (m->d_pexp) (void)hipFree(m->d_pexp);
  if (m->d_vexp) (void)hipFree(m->d_vexp);
  if (m->d_gexp) (void)hipFree(m->d_gexp);
  if (m->d_scratch) (void)hipFree(m->d_scratch);
  if (m->cg_exec) (void)hipGraphExecDestroy(m->cg_exec);
  if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
  if (m->cg_host) (void)hipHostFree(m->cg_host);
  for (hipEvent_t e : m->cg_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &pair : m->time_ev)
    for (hipEvent_t e : pair)
      if (e) (void)hipEventDestroy(e);
  delete m;
}

int64_t nqs_n_params(const nqs_model *m) { return m ? n_params_of(m) : -1; }

nqs_status nqs_chain_init(nqs_model *m, int8_t *chain_sigma, int32_t n_chains, uint64_t seed,
                          int32_t chain_offset, void *stream) {
  if (!m || !chain_sigma || n_chains < 1 || chain_offset < 0) return NQS_EINVAL;
  return dev(launch_chain_init(m, chain_sigma, n_chains, seed, chain_offset,
                               (hipStream_t)stream));
}

nqs_status nqs_sample(nqs_model *m, const void *params, int8_t *chain_sigma, int32_t n_chains,
                      int32_t n_sweeps, int32_t n_discard, uint64_t seed, uint64_t counter,
                      int32_t chain_offset, int8_t *samples, int64_t *n_accepted, void *eloc,
                      void *stream) {
  if (!m || !params || !chain_sigma || !samples || n_chains < 1 || n_sweeps < 1 ||
      n_discard < 0 || chain_offset < 0)
    return NQS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (m->ff.L) {
    hipError_t e = launch_ff_tables(m, params, st);
    if (e == hipSuccess)
      e = launch_ff_sweep(m, params, chain_sigma, n_chains, n_sweeps, n_discard, seed, counter,
                          chain_offset, samples, n_accepted, st);
    if (e == hipSuccess && eloc)
      e = launch_ff_local_energy(m, params, samples, int64_t(n_sweeps) * n_chains, eloc, st);
    return dev(e);
  }
  // With fewer than 16 chains per compute unit (at most one wavefront per SIMD pair) the
  // sweep is latency-bound and local energies are cheaper as a separate full-occupancy
  // pass over the recorded samples; with many chains they are fused into the sweep, unless
  // the sweep holds more than 4 hidden units per lane (its registers then leave room for
  // one wavefront per SIMD, and the separate pass is faster).
  const bool fuse = eloc && int64_t(n_chains) >= 16 * int64_t(m->cu_count) &&
                    (m->M + 63) / 64 <= 4;
  const int64_t n = int64_t(n_sweeps) * n_chains;
  // one scratch buffer serves the wide sweep's chain angles, then the local energies
  size_t need = sweep_scratch_bytes(m, n_chains);
  if (eloc && !fuse && grad_scratch_bytes(m, n) > need) need = grad_scratch_bytes(m, n);
  if (need) {
    nqs_status s = ensure_scratch(m, need);
    if (s != NQS_OK) return s;
  }
  hipError_t e;
  params = model_params(m, params, st, &e);
  if (e == hipSuccess) e = launch_tables(m, params, st);
  if (e == hipSuccess)
    e = launch_sweep(m, chain_sigma, n_chains, n_sweeps, n_discard, seed, counter, chain_offset,
                     samples, n_accepted, fuse ? eloc : nullptr,
                     sweep_scratch_bytes(m, n_chains) ? m->d_scratch : nullptr, st);
  if (e == hipSuccess && eloc && !fuse) {
    e = launch_theta_tanh(m, samples, n, m->d_scratch, false, st);
    if (e == hipSuccess)
      e = launch_local_energy(m, samples, grad_buffers(m, n, m->d_scratch).Tm, n, eloc, st);
  }
  return dev(e);
}

nqs_status nqs_sample_pt(nqs_model *m, const void *params, int8_t *chain_sigma,
                         int32_t *temp_index, int32_t n_chains, int32_t n_replicas,
                         int32_t n_sweeps, int32_t n_discard, uint64_t seed, uint64_t counter,
                         int32_t chain_offset, int8_t *samples, int64_t *n_accepted,
                         int64_t *n_swaps, void *eloc, void *stream) {
  if (!m || !params || !chain_sigma || !temp_index || !samples || n_chains < 1 ||
      n_replicas < 2 || n_replicas > 4 || n_sweeps < 1 || n_discard < 0 || chain_offset < 0 ||
      int64_t(n_chains) * n_replicas > INT32_MAX)
    return NQS_EINVAL;
  if (m->ff.L || !pt_supported(m)) return NQS_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = int64_t(n_sweeps) * n_chains;
  if (eloc) {
    nqs_status s = ensure_scratch(m, grad_scratch_bytes(m, n));
    if (s != NQS_OK) return s;
  }
  hipError_t e;
  params = model_params(m, params, st, &e);
  if (e == hipSuccess) e = launch_tables(m, params, st);
  const PtArgs pt{n_replicas, temp_index, n_swaps};
  if (e == hipSuccess)
    e = launch_sweep(m, chain_sigma, n_chains * n_replicas, n_sweeps, n_discard, seed, counter,
                     chain_offset, samples, n_accepted, nullptr, nullptr, st, &pt);
  if (e == hipSuccess && eloc) {
    e = launch_theta_tanh(m, samples, n, m->d_scratch, false, st);
    if (e == hipSuccess)
      e = launch_local_energy(m, samples, grad_buffers(m, n, m->d_scratch).Tm, n, eloc, st);
  }
  return dev(e);
}

nqs_status nqs_log_psi(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                       void *logpsi, void *stream) {
  if (!m || !params || n < 0 || (n > 0 && (!sigma || !logpsi))) return NQS_EINVAL;
  if (n == 0) return NQS_OK;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (m->ff.L) {
    e = launch_ff_tables(m, params, st);
    if (e == hipSuccess) e = launch_ff_log_psi(m, params, sigma, n, logpsi, st);
    return dev(e);
  }
  params = model_params(m, params, st, &e);
  if (e == hipSuccess) e = launch_tables(m, params, st);
  if (e == hipSuccess) e = launch_log_psi(m, sigma, n, logpsi, st);
  return dev(e);
}

nqs_status nqs_local_energy(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                            void *eloc, void *stream) {
  if (!m || !params || n < 0 || (n > 0 && (!sigma || !eloc))) return NQS_EINVAL;
  if (n == 0) return NQS_OK;
  hipStream_t st = (hipStream_t)stream;
  if (m->ff.L) {
    hipError_t e = launch_ff_tables(m, params, st);
    if (e == hipSuccess) e = launch_ff_local_energy(m, params, sigma, n, eloc, st);
    return dev(e);
  }
  nqs_status s = ensure_scratch(m, grad_scratch_bytes(m, n));
  if (s != NQS_OK) return s;
  hipError_t e;
  params = model_params(m, params, st, &e);
  if (e == hipSuccess) e = launch_tables(m, params, st);
  if (e == hipSuccess) e = launch_theta_tanh(m, sigma, n, m->d_scratch, false, st);
  time_begin(m, NQS_TIME_ELOC);
  time_mark(m, NQS_TIME_ELOC, 0, st);
  if (e == hipSuccess)
    e = launch_local_energy(m, sigma, grad_buffers(m, n, m->d_scratch).Tm, n, eloc, st);
  time_mark(m, NQS_TIME_ELOC, 1, st);
  return dev(e);
}

// the Jacobian products of nqs_log_psi_grad with the given scratch (grad_scratch_bytes)
// (symmetric RBM: the products of the expanded RBM, with the direction expanded before the
// JVP and the VJP summed over the symmetry copies after it)
static nqs_status log_psi_grad_with(nqs_model *m, const void *params, const int8_t *sigma,
                                    int64_t n, const void *u, void *vjp, const void *v,
                                    void *jvp, void *scr, hipStream_t st) {
  hipError_t e;
  params = model_params(m, params, st, &e);
  if (e == hipSuccess) e = launch_tables(m, params, st);
  if (e == hipSuccess) e = launch_theta_tanh(m, sigma, n, scr, true, st);
  if (e == hipSuccess && u && vjp) {
    e = launch_vjp_partials(m, sigma, n, (const double *)u, scr, nullptr, st);
    double *out = m->G ? m->d_gexp : (double *)vjp;
    if (e == hipSuccess) e = launch_vjp_reduce(m, n, scr, out, nullptr, st);
    if (e == hipSuccess && m->G) e = launch_symm_reduce(m, m->d_gexp, (double *)vjp, st);
  }
  if (e == hipSuccess && v && jvp) {
    if (m->G) {
      e = launch_symm_expand_dir(m, (const double *)v, m->d_vexp, nullptr, st);
      v = m->d_vexp;
    }
    if (e == hipSuccess) e = launch_prep_dir(m, v, scr, true, st);
    if (e == hipSuccess) e = launch_jvp(m, sigma, n, scr, (double *)jvp, nullptr, nullptr, st);
  }
  return dev(e);
}

// argument checks shared by both Jacobian entry points; n == 0 is answered here (vjp = 0)
static nqs_status log_psi_grad_args(nqs_model *m, const void *params, const int8_t *sigma,
                                    int64_t n, const void *u, void *vjp, const void *v,
                                    void *jvp, hipStream_t st, bool *done) {
  *done = true;
  if (!m || !params || n < 0 || (n > 0 && !sigma)) return NQS_EINVAL;
  const bool want_vjp = u && vjp, want_jvp = v && jvp;
  if (!want_vjp && !want_jvp) return NQS_EINVAL;
  if (n == 0) {
    const int cs = m->is_complex ? 2 : 1;
    if (want_vjp)
      hipLaunchKernelGGL(k_zero, dim3(grid_for(n_params_of(m) * cs)), dim3(256), 0, st,
                         n_params_of(m) * cs, (double *)vjp);
    return dev(hipGetLastError());
  }
  *done = false;
  return NQS_OK;
}

nqs_status nqs_log_psi_grad(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                            const void *u, void *vjp, const void *v, void *jvp, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  bool done;
  nqs_status s = log_psi_grad_args(m, params, sigma, n, u, vjp, v, jvp, st, &done);
  if (done) return s;
  if (m->ff.L) {
    s = ensure_scratch(m, ff_grad_scratch_bytes(m, n));
    if (s != NQS_OK) return s;
    time_begin(m, NQS_TIME_SV);   // the network's products: one timing pair per launcher
    hipError_t e = launch_ff_tables(m, params, st);
    if (e == hipSuccess) e = launch_ff_fb(m, params, sigma, n, m->d_scratch, st);
    if (e == hipSuccess && u && vjp)
      e = launch_ff_vjp(m, sigma, n, (const double *)u, m->d_scratch, (double *)vjp, nullptr, st);
    if (e == hipSuccess && v && jvp)
      e = launch_ff_jvp(m, params, sigma, n, (const double *)v, m->d_scratch, (double *)jvp,
                        nullptr, nullptr, st);
    return dev(e);
  }
  s = ensure_scratch(m, grad_scratch_bytes(m, n));
  if (s != NQS_OK) return s;
  return log_psi_grad_with(m, params, sigma, n, u, vjp, v, jvp, m->d_scratch, st);
}

nqs_status nqs_log_psi_grad_noalloc(nqs_model *m, const void *params, const int8_t *sigma,
                                    int64_t n, const void *u, void *vjp, const void *v,
                                    void *jvp, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  bool done;
  nqs_status s = log_psi_grad_args(m, params, sigma, n, u, vjp, v, jvp, st, &done);
  if (done) return s;
  if (m->ff.L) return NQS_EUNSUPPORTED;
  if (grad_scratch_bytes(m, n) > kNoAllocScratchBytes) return NQS_ENOMEM;
  void *scr = nullptr;
  s = noalloc_scratch(&scr);
  if (s != NQS_OK) return s;
  return log_psi_grad_with(m, params, sigma, n, u, vjp, v, jvp, scr, st);
}


nqs_status nqs_target_cdf(nqs_model *m, const void *log_target, int64_t n_states, double *cdf,
                          void *stream) {
  if (!m || !log_target || !cdf || n_states < 1) return NQS_EINVAL;
  return dev(launch_target_cdf(m, log_target, n_states, cdf, (hipStream_t)stream));
}

nqs_status nqs_target_draw(nqs_model *m, const double *cdf, int64_t n_states,
                           const int8_t *states, const void *log_target, int64_t n,
                           uint64_t seed, uint64_t counter, int8_t *sigma, void *log_target_out,
                           int64_t *index, void *stream) {
  if (!m || !cdf || !states || !log_target || n_states < 1 || n < 0 ||
      (n > 0 && (!sigma || !log_target_out)))
    return NQS_EINVAL;
  if (n == 0) return NQS_OK;
  return dev(launch_target_draw(m, cdf, n_states, states, log_target, n, seed, counter, sigma,
                                log_target_out, index, (hipStream_t)stream));
}

nqs_status nqs_overlap_step(nqs_model *m, void *params, const int8_t *sigma,
                            const void *log_target, int64_t n, double lr,
                            nqs_overlap_info *info, void *stream) {
  if (!m || !params || !sigma || !log_target || n < 1 || !isfinite(lr)) return NQS_EINVAL;
  nqs_status s = ensure_scratch(m, overlap_scratch_bytes(m, n));
  if (s != NQS_OK) return s;
  return overlap_step_impl(m, params, sigma, log_target, n, lr, m->d_scratch, info,
                           (hipStream_t)stream);
}

size_t nqs_sr_workspace_bytes(nqs_model *m, int64_t n) {
  if (!m || n < 2) return 0;
  return sr_workspace_bytes(m, n);
}

static bool sr_args_ok(const nqs_model *m, const void *params, const int8_t *sigma,
                       const void *eloc, const void *workspace, int64_t n, int32_t n_chains,
                       double lr, double diag_shift, double cg_tol, int32_t cg_maxiter) {
  return m && params && sigma && eloc && workspace && n >= 2 && cg_maxiter >= 1 &&
         cg_tol >= 0 && diag_shift >= 0 && isfinite(lr) && n_chains >= 0 && n_chains != 1 &&
         n_chains <= n && (n_chains == 0 || n % n_chains == 0);
}

nqs_status nqs_sr_step(nqs_model *m, void *params, const int8_t *sigma, const void *eloc,
                       int64_t n, int32_t n_chains, double lr, double diag_shift, double cg_tol,
                       int32_t cg_maxiter, void *workspace, size_t ws_bytes,
                       nqs_sr_info *info, void *stream) {
  if (!sr_args_ok(m, params, sigma, eloc, workspace, n, n_chains, lr, diag_shift, cg_tol,
                  cg_maxiter))
    return NQS_EINVAL;
  return sr_step_impl(m, params, sigma, eloc, n, n_chains, lr, diag_shift, cg_tol, cg_maxiter,
                      workspace, ws_bytes, info, false, (hipStream_t)stream);
}

nqs_status nqs_sr_step_async(nqs_model *m, void *params, const int8_t *sigma, const void *eloc,
                             int64_t n, int32_t n_chains, double lr, double diag_shift,
                             double cg_tol, int32_t cg_maxiter, void *workspace,
                             size_t ws_bytes, nqs_sr_info *info, void *stream) {
  if (!info || !sr_args_ok(m, params, sigma, eloc, workspace, n, n_chains, lr, diag_shift,
                           cg_tol, cg_maxiter))
    return NQS_EINVAL;
  return sr_step_impl(m, params, sigma, eloc, n, n_chains, lr, diag_shift, cg_tol, cg_maxiter,
                      workspace, ws_bytes, info, true, (hipStream_t)stream);
}

nqs_status nqs_sr_prepare(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                          void *workspace, size_t ws_bytes, void *stream) {
  if (!m || !params || !sigma || !workspace || n < 2) return NQS_EINVAL;
  if (m->ff.L) return NQS_EUNSUPPORTED;
  return sr_prepare_impl(m, params, sigma, n, workspace, ws_bytes, (hipStream_t)stream);
}

nqs_status nqs_sr_matvec(nqs_model *m, const int8_t *sigma, int64_t n, void *workspace,
                         size_t ws_bytes, const void *v, double diag_shift, void *out,
                         void *stream) {
  if (!m || !sigma || !workspace || !v || !out || n < 2 || !(diag_shift >= 0))
    return NQS_EINVAL;
  if (m->ff.L) return NQS_EUNSUPPORTED;
  return sr_matvec_impl(m, sigma, n, workspace, ws_bytes, v, diag_shift, out,
                        (hipStream_t)stream);
}

nqs_status nqs_autotune(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                        void *workspace, size_t ws_bytes, nqs_tune_report *report,
                        void *stream) {
  if (!m || !params || !sigma || !workspace || n < 2) return NQS_EINVAL;
  if (m->ff.L) return NQS_EUNSUPPORTED;
  return autotune_impl(m, params, sigma, n, workspace, ws_bytes, report, (hipStream_t)stream);
}

nqs_status nqs_set_cg_graphs(nqs_model *m, int32_t enable) {
  if (!m) return NQS_EINVAL;
  m->cg_graphs = enable != 0;
  return NQS_OK;
}

nqs_status nqs_time_kernel(nqs_model *m, int32_t what) {
  if (!m || what < NQS_TIME_NONE || what > NQS_TIME_ELOC) return NQS_EINVAL;
  for (auto &pair : m->time_ev)
    for (hipEvent_t &e : pair)
      if (!e && hipEventCreate(&e) != hipSuccess) return NQS_EDEVICE;
  m->time_what = what;
  m->time_n = 0;
  return NQS_OK;
}

nqs_status nqs_kernel_ms(nqs_model *m, float *ms) {
  if (!m || !ms || m->time_n < 1) return NQS_EINVAL;
  double total = 0.0;
  for (int k = 0; k < m->time_n; ++k) {
    float t = 0.f;
    if (hipEventSynchronize(m->time_ev[k][1]) != hipSuccess ||
        hipEventElapsedTime(&t, m->time_ev[k][0], m->time_ev[k][1]) != hipSuccess)
      return NQS_EDEVICE;
    total += t;
  }
  *ms = float(total);
  return NQS_OK;
}

nqs_status nqs_kernel_times(nqs_model *m, float *ms, int32_t cap, int32_t *count) {
  if (!m || !ms || !count || cap < 1 || m->time_n < 1) return NQS_EINVAL;
  const int k_end = m->time_n < cap ? m->time_n : cap;
  for (int k = 0; k < k_end; ++k) {
    float t = 0.f;
    if (hipEventSynchronize(m->time_ev[k][1]) != hipSuccess ||
        hipEventElapsedTime(&t, m->time_ev[k][0], m->time_ev[k][1]) != hipSuccess)
      return NQS_EDEVICE;
    ms[k] = t;
  }
  *count = k_end;
  return NQS_OK;
}

nqs_status nqs_set_sv_shape(nqs_model *m, int32_t pairs) {
  if (!m || (pairs != 2 && pairs != 4)) return NQS_EINVAL;
  m->sv_pairs = pairs;
  return NQS_OK;
}

}  // extern "C"
