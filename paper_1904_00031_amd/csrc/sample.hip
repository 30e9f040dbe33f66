// Parameter tables, chain initialisation, Metropolis sweeps, local energies and log psi.
//
// RBM (Sec. 2.2.2): log psi(s) = sum_i a_i s_i + sum_j ln cosh theta_j,
// theta_j = b_j + sum_i W_ji s_i. Moving from s to s' changes theta by delta_j, and
//   psi(s')/psi(s) = exp(sum_i a_i (s'_i - s_i)) * prod_j cosh(theta_j + delta_j)/cosh(theta_j)
//                  = exp(...) * prod_j [cosh(delta_j) + tanh(theta_j) sinh(delta_j)].
// A flip of site i (spin s) has delta_j = -2 s W_ji; an exchange on bond (i, k) with
// s_k = -s has delta_j = -2 s (W_ji - W_jk). cosh/sinh of 2 W_ji and of 2 (W_ji - W_jk)
// do not depend on the configuration, so they are tabulated once per call and each ratio
// term costs one complex multiply-add, with no transcendental function.
#include <string.h>

#include <type_traits>

#include "internal.hpp"

namespace {

// ---------------------------------------------------------------------------------
// Tables: one thread per element of the three index ranges
//   [0, N*M)            W transposed + flip tables
//   [N*M, N*M+Btot*M)   bond tables
//   then M + N + Btot   bias, a, a-factors
// ---------------------------------------------------------------------------------
template <typename T, bool C, typename PT>
__device__ __forceinline__ void tables_body(const DevModel &dm, const Tables<T> &tb,
                                            const PT *__restrict__ p, int quant, int need_flip,
                                            int need_bond, int bx, int gx) {
  const int N = dm.N, M = dm.M, B = dm.Btot;
  const int64_t nW = int64_t(N) * M, nB = int64_t(B) * M;
  const int64_t total = nW + nB + M + N + B;
  const int64_t offW = N + M;
  for (int64_t e = bx * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gx) * blockDim.x) {
    if (e < nW) {
      int i = int(e / M), j = int(e % M);
      V<double, C> w = vload<double, C>(p, offW + int64_t(j) * N + i);
      if (quant) {
        w.re = bf16_round(float(w.re));
        if (C) w.im = bf16_round(float(w.im));
      }
      vstore<T, C>(tb.Wt, int64_t(i) * M + j, vcast<double, C, T>(w));
      if (need_flip) {
        double x = 2 * w.re, y = 2 * w.im;
        double ch = cosh(x), sh = sinh(x), sy = 0, cy = 1;
        if (C) sincos(y, &sy, &cy);
        V<double, C> cc = vmake<double, C>(ch * cy, sh * sy);
        V<double, C> ss = vmake<double, C>(sh * cy, ch * sy);
        vstore<T, C>(tb.fC, int64_t(i) * M + j, vcast<double, C, T>(cc));
        vstore<T, C>(tb.fS, int64_t(i) * M + j, vcast<double, C, T>(ss));
      }
    } else if (e < nW + nB) {
      if (!need_bond) continue;
      int64_t q = e - nW;
      int b = int(q / M), j = int(q % M);
      int i = dm.bonds[2 * b], k = dm.bonds[2 * b + 1];
      V<double, C> wi = vload<double, C>(p, offW + int64_t(j) * N + i);
      V<double, C> wk = vload<double, C>(p, offW + int64_t(j) * N + k);
      if (quant) {
        wi.re = bf16_round(float(wi.re));
        wk.re = bf16_round(float(wk.re));
        if (C) {
          wi.im = bf16_round(float(wi.im));
          wk.im = bf16_round(float(wk.im));
        }
      }
      double x = 2 * (wi.re - wk.re), y = C ? 2 * (wi.im - wk.im) : 0.0;
      double ch = cosh(x), sh = sinh(x), sy = 0, cy = 1;
      if (C) sincos(y, &sy, &cy);
      V<double, C> cc = vmake<double, C>(ch * cy, sh * sy);
      V<double, C> ss = vmake<double, C>(sh * cy, ch * sy);
      vstore<T, C>(tb.bC, int64_t(b) * M + j, vcast<double, C, T>(cc));
      vstore<T, C>(tb.bS, int64_t(b) * M + j, vcast<double, C, T>(ss));
      if (tb.Wd && b < dm.B0) vstore<T, C>(tb.Wd, int64_t(b) * M + j, vcast<double, C, T>(vsub(wi, wk)));
    } else {
      int64_t q = e - nW - nB;
      if (q < M) {
        vstore<T, C>(tb.bv, q, vcast<double, C, T>(vload<double, C>(p, N + q)));
      } else if (q < M + N) {
        int i = int(q - M);
        V<double, C> a = vload<double, C>(p, i);
        tb.av[2 * i] = a.re;
        tb.av[2 * i + 1] = C ? a.im : 0.0;
        // exp(-2 s a_i): s = +1 -> row 0, s = -1 -> row 1
        for (int r = 0; r < 2; ++r) {
          double sgn = r == 0 ? -2.0 : 2.0;
          double mag = exp(sgn * a.re), sy = 0, cy = 1;
          if (C) sincos(sgn * a.im, &sy, &cy);
          tb.fa[2 * (int64_t(r) * N + i)] = mag * cy;
          tb.fa[2 * (int64_t(r) * N + i) + 1] = mag * sy;
        }
      } else {
        int b = int(q - M - N);
        int i = dm.bonds[2 * b], k = dm.bonds[2 * b + 1];
        V<double, C> ai = vload<double, C>(p, i), ak = vload<double, C>(p, k);
        double dr = ai.re - ak.re, di = C ? ai.im - ak.im : 0.0;
        for (int r = 0; r < 2; ++r) {
          double sgn = r == 0 ? -2.0 : 2.0;
          double mag = exp(sgn * dr), sy = 0, cy = 1;
          if (C) sincos(sgn * di, &sy, &cy);
          tb.ba[2 * (int64_t(r) * B + b)] = mag * cy;
          tb.ba[2 * (int64_t(r) * B + b) + 1] = mag * sy;
        }
      }
    }
  }
}

template <typename T, bool C, typename PT>
__global__ void k_tables(DevModel dm, Tables<T> tb, const PT *__restrict__ p, int quant,
                         int need_flip, int need_bond) {
  tables_body<T, C, PT>(dm, tb, p, quant, need_flip, need_bond, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------------
// Chain initialisation: Philox4x32-10, counter (chain, 0, site, TAG_INIT).
// ---------------------------------------------------------------------------------
__global__ void k_init_flip(int8_t *sig, int n_chains, int N, uint32_t k0, uint32_t k1,
                            uint32_t chain_offset) {
  int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= int64_t(n_chains) * N) return;
  int c = int(e / N), i = int(e % N);
  Philox4 w = philox4x32_10(chain_offset + uint32_t(c), 0u, uint32_t(i), TAG_INIT, k0, k1);
  sig[e] = (w.w[0] >> 31) == 0 ? int8_t(1) : int8_t(-1);
}

// zero magnetisation: N/2 up then N/2 down, shuffled by Fisher-Yates from the last site
__global__ void k_init_sz0(int8_t *sig, int n_chains, int N, uint32_t k0, uint32_t k1,
                           uint32_t chain_offset) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_chains) return;
  int8_t *row = sig + int64_t(c) * N;
  for (int i = 0; i < N; ++i) row[i] = i < N / 2 ? int8_t(1) : int8_t(-1);
  for (int k = N - 1; k >= 1; --k) {
    Philox4 w = philox4x32_10(chain_offset + uint32_t(c), 0u, uint32_t(k), TAG_INIT, k0, k1);
    int r = rng_index(w.w[0], uint32_t(k + 1));
    int8_t t = row[k];
    row[k] = row[r];
    row[r] = t;
  }
}

// ---------------------------------------------------------------------------------
// Local energy of one configuration (Eq. 5), evaluated by one wavefront whose lane l
// holds t_j = tanh(theta_j) for j = l + 64 r (r < R) in registers; the spins are in LDS.
// Connected configurations (every site for TFIM, every anti-aligned bond with a nonzero
// coupling for Heisenberg) are enumerated as a wave-uniform bit mask; for each one the
// lanes form their ratio terms C_row,j - s t_j S_row,j from the row-major tables (LDS
// when staged) and a DPP complex product gives psi(s')/psi(s) up to the visible-bias
// factor. Accumulates in double; returns (re, im) on every lane.
// ---------------------------------------------------------------------------------
template <typename T, bool C, int R, bool TL>
__device__ __forceinline__ void eloc_regs(const DevModel &dm, const Tables<T> &tb,
                                          const int8_t *sig, const V<T, C> *t, int lane,
                                          const T *lCe, const T *lSe, double &out_re,
                                          double &out_im) {
  const int N = dm.N, M = dm.M, B = dm.Btot;
  const bool tfim = dm.ham == NQS_TFIM;
  const T *gCe = tfim ? tb.fC : tb.bC;
  const T *gSe = tfim ? tb.fS : tb.bS;
  double diag = 0.0;
  for (int b = lane; b < B; b += 64)
    diag += dm.bond_diag[b] * double(sig[dm.bonds[2 * b]]) * double(sig[dm.bonds[2 * b + 1]]);
  double er = 0.0, ei = 0.0;
  const int ncand = tfim ? (dm.h != 0.0 ? N : 0) : B;
  for (int c0 = 0; c0 < ncand; c0 += 64) {
    // bit q of `mask`: configuration c0 + q is connected; bit q of `up`: its spin s = +1
    const int c = c0 + lane;
    bool on = false, sup = false;
    if (c < ncand) {
      if (tfim) {
        on = true;
        sup = sig[c] > 0;
      } else {
        const int si = sig[dm.bonds[2 * c]], sk = sig[dm.bonds[2 * c + 1]];
        on = si != sk && dm.bond_off[c] != 0.0;
        sup = si > 0;
      }
    }
    uint64_t mask = __ballot(on);
    const uint64_t up = __ballot(sup);
    while (mask) {
      const int q = __builtin_ctzll(mask);
      mask &= mask - 1;
      const int row = c0 + q;
      const int s = ((up >> q) & 1) ? 1 : -1;
      const T ts = T(s);
      V<T, C> p = vmake<T, C>(T(1), T(0));
      int pe = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int j = lane + 64 * r;
        if (j < M) {
          V<T, C> cc, ss;
          if constexpr (TL) {
            cc = vload<T, C>(lCe, int64_t(row) * M + j);
            ss = vload<T, C>(lSe, int64_t(row) * M + j);
          } else {
            cc = vload<T, C>(gCe, int64_t(row) * M + j);
            ss = vload<T, C>(gSe, int64_t(row) * M + j);
          }
          p = vmul(p, vsub(cc, vscale(vmul(t[r], ss), ts)));
        }
        if ((r & 3) == 3) vrenorm(p, pe);
      }
      vrenorm(p, pe);
      const V<T, C> w = wave_cprod_dpp(p, pe);
      const double el = tfim ? -dm.h : dm.bond_off[row];
      const double *af = tfim ? tb.fa + 2 * (int64_t(s > 0 ? 0 : 1) * N + row)
                              : tb.ba + 2 * (int64_t(s > 0 ? 0 : 1) * B + row);
      const double rr = ldexp(double(w.re), pe), ri = C ? ldexp(double(w.im), pe) : 0.0;
      er += el * (rr * af[0] - ri * af[1]);
      ei += el * (rr * af[1] + ri * af[0]);
    }
  }
  out_re = wave_sum_dpp(diag) + er;
  out_im = C ? ei : 0.0;
}

// ---------------------------------------------------------------------------------
// Local energy with four connected configurations per pass (M <= 256): the 16 lanes of
// DPP row g take configuration g of the pass, each lane multiplies the ratio terms of
// hidden units j = lane%16 + 16 q (t_j read from LDS), and a 4-step DPP product inside
// the row finishes each ratio. Same result as eloc_regs, a quarter of the reductions.
// ---------------------------------------------------------------------------------
template <typename T, bool C, bool TL, int TP>
__device__ __forceinline__ void eloc_grouped(const DevModel &dm, const Tables<T> &tb,
                                             const int8_t *sig, const T *tj, int lane,
                                             const T *lCe, const T *lSe, double &out_re,
                                             double &out_im) {
  const int N = dm.N, M = dm.M, B = dm.Btot;
  const bool tfim = dm.ham == NQS_TFIM;
  const T *gCe = tfim ? tb.fC : tb.bC;
  const T *gSe = tfim ? tb.fS : tb.bS;
  const int lo = lane & 15, g = lane >> 4;
  // the lane's t_j (j = lo + 16 q) for every pass, loaded once
  V<T, C> tv[TP];
#pragma unroll
  for (int q = 0; q < TP; ++q)
    tv[q] = lo + 16 * q < M ? vload<T, C>(tj, lo + 16 * q) : vmake<T, C>(T(0), T(0));
  double diag = 0.0;
  for (int b = lane; b < B; b += 64)
    diag += dm.bond_diag[b] * double(sig[dm.bonds[2 * b]]) * double(sig[dm.bonds[2 * b + 1]]);
  double er = 0.0, ei = 0.0;
  const int ncand = tfim ? (dm.h != 0.0 ? N : 0) : B;
  for (int c0 = 0; c0 < ncand; c0 += 64) {
    const int c = c0 + lane;
    bool on = false, sup = false;
    if (c < ncand) {
      if (tfim) {
        on = true;
        sup = sig[c] > 0;
      } else {
        const int si = sig[dm.bonds[2 * c]], sk = sig[dm.bonds[2 * c + 1]];
        on = si != sk && dm.bond_off[c] != 0.0;
        sup = si > 0;
      }
    }
    uint64_t mask = __ballot(on);
    const uint64_t up = __ballot(sup);
    while (mask) {
      int q4[4], cnt = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        q4[u] = -1;
        if (mask) {
          q4[u] = __builtin_ctzll(mask);
          mask &= mask - 1;
          ++cnt;
        }
      }
      const int myq = g == 0 ? q4[0] : (g == 1 ? q4[1] : (g == 2 ? q4[2] : q4[3]));
      V<T, C> p = vmake<T, C>(T(1), T(0));
      int pe = 0;
      if (myq >= 0) {
        const int row = c0 + myq;
        const T ts = ((up >> myq) & 1) ? T(1) : T(-1);
        V<T, C> cc[TP], ss[TP];
#pragma unroll
        for (int q = 0; q < TP; ++q) {
          const int j = lo + 16 * q < M ? lo + 16 * q : 0;
          if constexpr (TL) {
            cc[q] = vload<T, C>(lCe, int64_t(row) * M + j);
            ss[q] = vload<T, C>(lSe, int64_t(row) * M + j);
          } else {
            cc[q] = vload<T, C>(gCe, int64_t(row) * M + j);
            ss[q] = vload<T, C>(gSe, int64_t(row) * M + j);
          }
        }
#pragma unroll
        for (int q = 0; q < TP; ++q) {
          if (lo + 16 * q < M) p = vmul(p, vsub(cc[q], vscale(vmul(tv[q], ss[q]), ts)));
          if ((q & 3) == 3) vrenorm(p, pe);
        }
      }
      vrenorm(p, pe);
      cprod_step<T, C, DPP_QP_XOR1>(p, pe);
      cprod_step<T, C, DPP_QP_XOR2>(p, pe);
      cprod_step<T, C, DPP_ROR4>(p, pe);
      cprod_step<T, C, DPP_ROR8>(p, pe);
      vrenorm(p, pe);
      for (int u = 0; u < cnt; ++u) {
        const int row = c0 + q4[u];
        const int s = ((up >> q4[u]) & 1) ? 1 : -1;
        const double wr = double(readlane_v(p.re, 16 * u));
        const double wi = C ? double(readlane_v(p.im, 16 * u)) : 0.0;
        const int we = __builtin_amdgcn_readlane(pe, 16 * u);
        const double el = tfim ? -dm.h : dm.bond_off[row];
        const double *af = tfim ? tb.fa + 2 * (int64_t(s > 0 ? 0 : 1) * N + row)
                                : tb.ba + 2 * (int64_t(s > 0 ? 0 : 1) * B + row);
        const double rr = ldexp(wr, we), ri = ldexp(wi, we);
        er += el * (rr * af[0] - ri * af[1]);
        ei += el * (rr * af[1] + ri * af[0]);
      }
    }
  }
  out_re = wave_sum_dpp(diag) + er;
  out_im = C ? ei : 0.0;
}

// ---------------------------------------------------------------------------------
// Metropolis sweeps. One chain per wavefront; lane l owns hidden units l + 64 r (r < R):
// theta_j cached in double (exact running sums of +/-2 W), t_j = tanh(theta_j) in T.
// A proposal costs R ratio terms per lane (C - s t S), a DPP product reduction carried as
// mantissa x 2^exponent, and a wave-uniform accept decision in double. On acceptance
// theta moves by -2 s W_row and t by the addition formula t' = (C t - s S) / term, whose
// denominator is the ratio term already computed; t is recomputed from theta at the end
// of every sweep, so rounding does not accumulate over sweeps. Spins live in LDS. When
// TL, the C/S rows of every connected configuration (which then include the move rows)
// and the W rows of the moves are staged in LDS; otherwise they are read from global
// memory, with the next proposal's rows fetched one step ahead for small R (the
// counter-based stream makes the next proposal known). Float models with more than four
// units per lane and tables in global memory run k_sweep_wide instead. After each recorded sweep the
// chain's local energy is evaluated from its cached t.
// ---------------------------------------------------------------------------------
constexpr int kMaxReplicas = 4;   // replicas are the (at most 4) wavefronts of a block
struct SweepArgs {
  int8_t *chain_sigma;
  int n_chains, n_sweeps, n_discard;
  uint32_t k0, k1, counter, chain_offset;
  int8_t *samples;
  int64_t *n_acc;
  double *eloc;
  int cs_rows;       // C/S rows staged when TL (N for TFIM, Btot for Heisenberg)
  int w_rows;        // W rows of the moves (N for flips, B0 for exchanges)
  int wave_bytes;    // per-wavefront LDS: spins (Npad bytes), then t (M values)
  int Npad;
  // parallel tempering (n_rep > 1): a block holds one tempered chain, wavefront w its
  // replica w; chain rows, proposal streams and n_acc are per replica (chain c R + w);
  // temp holds the temperature index of every replica [C R] (in/out), n_swap [C] the
  // accepted exchanges, group_offset the first chain index of the swap streams
  int n_rep;
  int *temp;
  int64_t *n_swap;
  uint32_t group_offset;
  double betas[kMaxReplicas];
};

// whether the wavefront's sum of x exceeds th, the same on every lane: row sums by DPP,
// rows combined by the row broadcasts (lane 63 ends with (rows 0 + 1) + (rows 2 + 3)),
// and one compare on lane 63
__device__ __forceinline__ int wave_sum_gt(float x, float th) {
  x += dpp_v<DPP_QP_XOR1>(x);
  x += dpp_v<DPP_QP_XOR2>(x);
  x += dpp_v<DPP_ROR4>(x);
  x += dpp_v<DPP_ROR8>(x);
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), DPP_BCAST15, 0xA, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), DPP_BCAST31, 0xC, 0xF, false));
  return int((__ballot(x > th) >> 63) & 1ull);
}

// SM: N <= 64, the spins also held as a wave-uniform bit mask (bit i set: spin i up), so
// the spins of a proposal and their update are scalar bit operations. FE: the fused local
// energy is compiled in (the single-model sweep fuses it only with at most four hidden
// units per lane; leaving it out of the other shapes frees their registers)
template <typename T, bool C, int R, bool TL, bool SM, bool FE = true>
__device__ __forceinline__ void sweep_block(const DevModel &dm, const Tables<T> &tb,
                                            const SweepArgs &a, int chain_base) {
  extern __shared__ __align__(16) unsigned char lds_u8[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int chain = __builtin_amdgcn_readfirstlane(chain_base + wid);
  const int N = dm.N, M = dm.M;
  constexpr int cs = C ? 2 : 1;
  const bool flip = dm.move == NQS_MOVE_FLIP;
  const T *gC = flip ? tb.fC : tb.bC;
  const T *gS = flip ? tb.fS : tb.bS;
  const T *gW = flip ? tb.Wt : tb.Wd;
  T *lC = reinterpret_cast<T *>(lds_u8);
  T *lS = lC + int64_t(a.cs_rows) * M * cs;
  T *lW = lS + int64_t(a.cs_rows) * M * cs;
  const int64_t tab_bytes =
      TL ? (int64_t(2) * a.cs_rows + a.w_rows) * M * cs * int64_t(sizeof(T)) : 0;
  if constexpr (TL) {
    const T *gCe = dm.ham == NQS_TFIM ? tb.fC : tb.bC;
    const T *gSe = dm.ham == NQS_TFIM ? tb.fS : tb.bS;
    const int64_t ce = int64_t(a.cs_rows) * M * cs, we = int64_t(a.w_rows) * M * cs;
    for (int64_t e = threadIdx.x; e < ce; e += blockDim.x) {
      lC[e] = gCe[e];
      lS[e] = gSe[e];
    }
    for (int64_t e = threadIdx.x; e < we; e += blockDim.x) lW[e] = gW[e];
  }
  // |visible-bias factor|^2 of every row for either spin and the color-0 bonds, staged
  // once per block after the wavefronts' regions: every sweep's proposal draw reads them
  const int afn = flip ? N : dm.Btot;
  const int64_t aux_off =
      (tab_bytes + int64_t(blockDim.x >> 6) * a.wave_bytes + 15) & ~int64_t(15);
  double *la2 = reinterpret_cast<double *>(lds_u8 + aux_off);  // [2][afn]
  int *lbond = reinterpret_cast<int *>(la2 + 2 * afn);           // [B0][2]
  {
    const double *afb = flip ? tb.fa : tb.ba;
    for (int e = threadIdx.x; e < 2 * afn; e += blockDim.x)
      la2[e] = afb[2 * e] * afb[2 * e] + afb[2 * e + 1] * afb[2 * e + 1];
    if (!flip)
      for (int e = threadIdx.x; e < 2 * dm.B0; e += blockDim.x) lbond[e] = dm.bonds[e];
  }
  // parallel tempering: the replicas' 2 Re log psi and temperature indices after the
  // auxiliary tables
  const bool pt = a.n_rep > 1;
  const int64_t pt_off = (aux_off + int64_t(16) * afn + (flip ? 0 : int64_t(8) * dm.B0) + 15) &
                         ~int64_t(15);
  double *ptL = reinterpret_cast<double *>(lds_u8 + pt_off);   // [R]
  int *ptT = reinterpret_cast<int *>(ptL + kMaxReplicas);      // [R]
  if (pt && lane == 0) ptT[wid] = a.temp[chain];
  __syncthreads();
  if (chain >= a.n_chains) return;
  // inverse temperature of this replica (1 without tempering)
  double beta = pt ? a.betas[ptT[wid]] : 1.0;
  int64_t n_swaps = 0;
  int8_t *sig = reinterpret_cast<int8_t *>(lds_u8 + tab_bytes + int64_t(wid) * a.wave_bytes);
  T *tj = reinterpret_cast<T *>(lds_u8 + tab_bytes + int64_t(wid) * a.wave_bytes + a.Npad);
  for (int i = lane; i < N; i += 64) sig[i] = a.chain_sigma[int64_t(chain) * N + i];
  wave_sync();

  auto row_ld = [&](const T *lp, const T *gp, int row, int j) __attribute__((always_inline)) -> V<T, C> {
    if constexpr (TL)
      return vload<T, C>(lp, int64_t(row) * M + j);
    else
      return vload<T, C>(gp, int64_t(row) * M + j);
  };

  double thr[R], thi[R];
  V<T, C> t[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = lane + 64 * r;
    thr[r] = 0.0;
    thi[r] = 0.0;
    t[r] = vmake<T, C>(T(0), T(0));
    if (j < M) {
      V<double, C> acc = vload<double, C>(tb.bv, j);
      for (int i = 0; i < N; ++i) {
        const double s = double(sig[i]);
        V<double, C> w = vload<double, C>(tb.Wt, int64_t(i) * M + j);
        acc.re += s * w.re;
        if (C) acc.im += s * w.im;
      }
      thr[r] = acc.re;
      thi[r] = C ? acc.im : 0.0;
      t[r] = vtanh<T, C>(vmake<T, C>(T(thr[r]), T(thi[r])));
    }
  }

  const uint32_t cid = a.chain_offset + uint32_t(chain);
  const int total = a.n_discard + a.n_sweeps;
  // spins mirrored in registers (lane l holds sites l, l+64, l+128, l+192) for N <= 256,
  // so that the spin of a proposed site is one readlane
  const bool sregs = !SM && N <= 256;
  int sp0 = 0, sp1 = 0, sp2 = 0, sp3 = 0;
  uint64_t smask = 0;
  if constexpr (SM) {
    smask = __ballot(lane < N && sig[lane] > 0);
  } else if (sregs) {
    sp0 = lane < N ? sig[lane] : 0;
    sp1 = lane + 64 < N ? sig[lane + 64] : 0;
    sp2 = lane + 128 < N ? sig[lane + 128] : 0;
    sp3 = lane + 192 < N ? sig[lane + 192] : 0;
  }
  // with few hidden units per lane the next proposal's rows are fetched one step ahead;
  // with many, the R independent loads of a step already overlap
  constexpr bool PF = R <= 4;
  struct Rows {
    V<T, C> c[R], s[R], w[R];
  };
  auto load_rows = [&](int row) __attribute__((always_inline)) -> Rows {
    Rows o;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = lane + 64 * r < M ? lane + 64 * r : 0;
      o.c[r] = row_ld(lC, gC, row, j);
      o.s[r] = row_ld(lS, gS, row, j);
      o.w[r] = row_ld(lW, gW, row, j);
    }
    return o;
  };
  int64_t acc_count = 0;
  for (int sw = 0; sw < total; ++sw) {
    for (int st0 = 0; st0 < N; st0 += 64) {
      // the random numbers of proposals st0 .. st0+63, one per lane: table row, the two
      // sites, the uniform, and |exp(visible-bias change)|^2 for either spin
      const int nst = N - st0 < 64 ? N - st0 : 64;
      int rowv = 0, iv = 0, kv = 0;
      double uv = 0.0, a2p = 0.0, a2m = 0.0;
      float thp = 0.f, thm = 0.f;  // log2(u) - log2|a-factor|^2, for the FP32 decision
      if (lane < nst) {
        const Philox4 w = philox4x32_10(cid, a.counter + uint32_t(sw), uint32_t(st0 + lane),
                                        TAG_PROPOSAL, a.k0, a.k1);
        if (flip) {
          iv = rng_index(w.w[0], uint32_t(N));
          rowv = iv;
          kv = iv;
        } else {
          rowv = rng_index(w.w[0], uint32_t(dm.B0));
          iv = lbond[2 * rowv];
          kv = lbond[2 * rowv + 1];
        }
        uv = rng_uniform(w.w[1], w.w[2]);
        a2p = la2[rowv];
        a2m = la2[afn + rowv];
        // |ratio|^(2 beta) > u  <=>  log2 |ratio|^2 > log2(u) / beta
        const float lu = pt ? float(double(__log2f(float(uv))) / beta) : __log2f(float(uv));
        thp = lu - __log2f(float(a2p));
        thm = lu - __log2f(float(a2m));
      }
      if constexpr (SM) {
        // one proposal; with prefetch, the rows of proposal l + 1 go to nxt (the loop
        // below alternates the two buffers, so no rows are copied)
        auto proposal = [&](int l, Rows &cur, Rows &nxt) __attribute__((always_inline)) {
          const int ic = __builtin_amdgcn_readlane(iv, l);
          const int kc = __builtin_amdgcn_readlane(kv, l);
          if constexpr (PF) {
            nxt = load_rows(__builtin_amdgcn_readlane(rowv, l + 1 < nst ? l + 1 : l));
          } else {
            if (l > 0) cur = load_rows(__builtin_amdgcn_readlane(rowv, l));
          }
          const int s = ((smask >> ic) & 1ull) ? 1 : -1;
          const int sk = flip ? -s : (((smask >> kc) & 1ull) ? 1 : -1);
          if (sk != s) {  // an exchange of equal spins is the identity move
            const T ts = T(s);
            V<T, C> term[R];
  #pragma unroll
            for (int r = 0; r < R; ++r) term[r] = vsub(cur.c[r], vscale(vmul(t[r], cur.s[r]), ts));
            // with few units per lane the updated t is formed before the decision (it
            // overlaps the reduction) and only selected after it
            V<T, C> tn[PF ? R : 1];
            if constexpr (PF) {
  #pragma unroll
              for (int r = 0; r < R; ++r)
                tn[r] = vdiv(vsub(vmul(cur.c[r], t[r]), vscale(cur.s[r], ts)), term[r]);
            }
            int accept;
            if constexpr (sizeof(T) == 4) {
              // log-domain decision: accept iff sum_j log2|term_j|^2 > log2(u) - log2|a|^2
              float lp = 0.f;
  #pragma unroll
              for (int r0 = 0; r0 < R; r0 += 4) {
                float pm = 1.f;
  #pragma unroll
                for (int r = r0; r < r0 + 4 && r < R; ++r)
                  if (lane + 64 * r < M) pm *= float(vabs2(term[r]));
                lp += __log2f(pm);
              }
              const float th = readlane_v(s > 0 ? thp : thm, l);
              accept = wave_sum_gt(lp, th);
            } else {
              T pm = T(1);
              int pe = 0;
  #pragma unroll
              for (int r = 0; r < R; ++r) {
                if (lane + 64 * r < M) pm *= vabs2(term[r]);
                if ((r & 3) == 3) {
                  int e;
                  pm = nfrexp(pm, &e);
                  pe += e;
                }
              }
              {
                int e;
                pm = nfrexp(pm, &e);
                pe += e;
              }
              const T pmw = wave_prod_dpp(pm, pe);
              const double a2 = readlane_v(s > 0 ? a2p : a2m, l);
              double q = ldexp(double(pmw), pe) * a2;
              if (pt && beta != 1.0) q = exp(beta * log(q));   // |psi'/psi|^(2 beta)
              const double u = readlane_v(uv, l);
              accept = __builtin_amdgcn_readfirstlane(int((q >= 1.0) || (u < q)));
            }
            if (accept) {
              // with few units per lane every lane updates (no branch on the lane; lanes past
              // M carry values that no sum reads and that the end of the sweep clears); with
              // many, the lane test keeps the register allocation of the update compact
  #pragma unroll
              for (int r = 0; r < R; ++r) {
                if (R <= 4 || lane + 64 * r < M) {
                  thr[r] -= 2.0 * double(s) * double(cur.w[r].re);
                  if (C) thi[r] -= 2.0 * double(s) * double(cur.w[r].im);
                  if constexpr (PF)
                    t[r] = tn[r];
                  else
                    t[r] = vdiv(vsub(vmul(cur.c[r], t[r]), vscale(cur.s[r], ts)), term[r]);
                }
              }
              smask ^= (1ull << ic) | (flip ? 0ull : (1ull << kc));
              if (lane == 0) {
                sig[ic] = int8_t(-s);
                if (!flip) sig[kc] = int8_t(s);
              }
              ++acc_count;
            }
          }
        };
        Rows ra = load_rows(__builtin_amdgcn_readlane(rowv, 0)), rb;
        if constexpr (PF) {
          int l = 0;
          for (; l + 1 < nst; l += 2) {
            proposal(l, ra, rb);
            proposal(l + 1, rb, ra);
          }
          if (l < nst) proposal(l, ra, rb);
        } else {
          for (int l = 0; l < nst; ++l) proposal(l, ra, rb);
        }
      } else {
        // the same proposal with the spins in registers or LDS (a plain loop: a closure
        // here made the compiler keep the chain state in scratch memory). Without the
        // prefetch, the rows of a move are read only once it is known not to be the
        // identity (an exchange of equal spins reads nothing).
        Rows cur;
        if constexpr (PF) cur = load_rows(__builtin_amdgcn_readlane(rowv, 0));
        for (int l = 0; l < nst; ++l) {
          const int ic = __builtin_amdgcn_readlane(iv, l);
          const int kc = __builtin_amdgcn_readlane(kv, l);
          Rows nxt;
          if constexpr (PF) nxt = load_rows(__builtin_amdgcn_readlane(rowv, l + 1 < nst ? l + 1 : l));
          int s, sk;
          if (sregs) {
            s = __builtin_amdgcn_readlane(ic < 64 ? sp0 : (ic < 128 ? sp1 : (ic < 192 ? sp2 : sp3)),
                                          ic & 63);
            sk = flip ? -s
                      : __builtin_amdgcn_readlane(
                            kc < 64 ? sp0 : (kc < 128 ? sp1 : (kc < 192 ? sp2 : sp3)), kc & 63);
          } else {
            s = __builtin_amdgcn_readfirstlane(int(sig[ic]));
            sk = flip ? -s : __builtin_amdgcn_readfirstlane(int(sig[kc]));
          }
          if (sk != s) {  // an exchange of equal spins is the identity move
          const T ts = T(s);
          int accept;
          if constexpr (!PF) cur = load_rows(__builtin_amdgcn_readlane(rowv, l));
          V<T, C> term[R];
#pragma unroll
          for (int r = 0; r < R; ++r) term[r] = vsub(cur.c[r], vscale(vmul(t[r], cur.s[r]), ts));
          // updated t formed before the decision for few units per lane (as above)
          V<T, C> tn[PF ? R : 1];
          if constexpr (PF) {
#pragma unroll
            for (int r = 0; r < R; ++r)
              tn[r] = vdiv(vsub(vmul(cur.c[r], t[r]), vscale(cur.s[r], ts)), term[r]);
          }
          if constexpr (sizeof(T) == 4) {
            // log-domain decision: accept iff sum_j log2|term_j|^2 > log2(u) - log2|a|^2
            float lp = 0.f;
#pragma unroll
            for (int r0 = 0; r0 < R; r0 += 4) {
              float pm = 1.f;
#pragma unroll
              for (int r = r0; r < r0 + 4 && r < R; ++r)
                if (lane + 64 * r < M) pm *= float(vabs2(term[r]));
              lp += __log2f(pm);
            }
            const float th = readlane_v(s > 0 ? thp : thm, l);
            accept = wave_sum_gt(lp, th);
          } else {
            T pm = T(1);
            int pe = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              if (lane + 64 * r < M) pm *= vabs2(term[r]);
              if ((r & 3) == 3) {
                int e;
                pm = nfrexp(pm, &e);
                pe += e;
              }
            }
            {
              int e;
              pm = nfrexp(pm, &e);
              pe += e;
            }
            const T pmw = wave_prod_dpp(pm, pe);
            const double a2 = readlane_v(s > 0 ? a2p : a2m, l);
            double q = ldexp(double(pmw), pe) * a2;
            if (pt && beta != 1.0) q = exp(beta * log(q));   // |psi'/psi|^(2 beta)
            const double u = readlane_v(uv, l);
            accept = __builtin_amdgcn_readfirstlane(int((q >= 1.0) || (u < q)));
          }
          if (accept) {
            // with few units per lane every lane updates (no branch on the lane; lanes past
            // M carry values that no sum reads and that the end of the sweep clears); with
            // many, the lane test keeps the register allocation of the update compact
#pragma unroll
            for (int r = 0; r < R; ++r) {
              if (R <= 4 || lane + 64 * r < M) {
                thr[r] -= 2.0 * double(s) * double(cur.w[r].re);
                if (C) thi[r] -= 2.0 * double(s) * double(cur.w[r].im);
                if constexpr (PF)
                  t[r] = tn[r];
                else
                  t[r] = vdiv(vsub(vmul(cur.c[r], t[r]), vscale(cur.s[r], ts)), term[r]);
              }
            }
          }
          if (accept) {
              // spin registers (one lane each) and the LDS copy
              if (sregs) {
                if (ic < 64)
                  sp0 = lane == (ic & 63) ? -s : sp0;
                else if (ic < 128)
                  sp1 = lane == (ic & 63) ? -s : sp1;
                else if (ic < 192)
                  sp2 = lane == (ic & 63) ? -s : sp2;
                else
                  sp3 = lane == (ic & 63) ? -s : sp3;
                if (!flip) {
                  if (kc < 64)
                    sp0 = lane == (kc & 63) ? s : sp0;
                  else if (kc < 128)
                    sp1 = lane == (kc & 63) ? s : sp1;
                  else if (kc < 192)
                    sp2 = lane == (kc & 63) ? s : sp2;
                  else
                    sp3 = lane == (kc & 63) ? s : sp3;
                }
              }
              if (lane == 0) {
                sig[ic] = int8_t(-s);
                if (!flip) sig[kc] = int8_t(s);
              }
              if (!sregs) wave_sync();
              ++acc_count;
            }
          }
          if constexpr (PF) cur = nxt;
        }
      }
    }
    wave_sync();
    // end of sweep: tanh from the exact angles (zero, with the angles, past M when the
    // accept update runs on every lane)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (lane + 64 * r < M) {
        t[r] = vtanh<T, C>(vmake<T, C>(T(thr[r]), T(thi[r])));
      } else if (R <= 4) {
        t[r] = vmake<T, C>(T(0), T(0));
        thr[r] = 0.0;
        thi[r] = 0.0;
      }
    }
    if (pt) {
      // exchanges of adjacent temperatures: every replica's L = 2 Re log psi in double from
      // its exact angles and spins, then one thread decides k = 0 .. R-2 in order
      double lr = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (lane + 64 * r < M) lr += vlncosh<double, C>(vmake<double, C>(thr[r], thi[r])).re;
      for (int i = lane; i < N; i += 64) lr += tb.av[2 * i] * double(sig[i]);
      lr = wave_sum_dpp(lr);
      if (lane == 0) ptL[wid] = 2.0 * lr;
      __syncthreads();
      if (threadIdx.x == 0) {
        const uint32_t gid = a.group_offset + uint32_t(chain / a.n_rep);
        for (int k = 0; k + 1 < a.n_rep; ++k) {
          int ia = 0, ib = 0;
          for (int q = 0; q < a.n_rep; ++q) {
            if (ptT[q] == k) ia = q;
            if (ptT[q] == k + 1) ib = q;
          }
          const double ex = (a.betas[k] - a.betas[k + 1]) * (ptL[ib] - ptL[ia]);
          const Philox4 w = philox4x32_10(gid, a.counter + uint32_t(sw), uint32_t(k), TAG_SWAP,
                                          a.k0, a.k1);
          const double u = rng_uniform(w.w[1], w.w[2]);
          if (ex >= 0.0 || u < exp(ex)) {
            ptT[ia] = k + 1;
            ptT[ib] = k;
            ++n_swaps;
          }
        }
      }
      __syncthreads();
      beta = a.betas[ptT[wid]];
    }
    if (sw >= a.n_discard && (!pt || ptT[wid] == 0)) {
      // tempering: only the replica holding beta = 1 records, as sample c of the sweep
      const int64_t smp = pt ? int64_t(sw - a.n_discard) * (a.n_chains / a.n_rep) + chain / a.n_rep
                             : int64_t(sw - a.n_discard) * a.n_chains + chain;
      int8_t *dst = a.samples + smp * N;
      for (int i = lane; i < N; i += 64) dst[i] = sig[i];
      if (FE && a.eloc) {
        double er, ei;
        if (M <= 256) {
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (lane + 64 * r < M) vstore<T, C>(tj, lane + 64 * r, t[r]);
          wave_sync();
          eloc_grouped<T, C, TL, (4 * R < 16 ? 4 * R : 16)>(dm, tb, sig, tj, lane, lC, lS, er, ei);
          wave_sync();
        } else {
          eloc_regs<T, C, R, TL>(dm, tb, sig, t, lane, lC, lS, er, ei);
        }
        if (lane == 0) {
          if (C) {
            a.eloc[2 * smp] = er;
            a.eloc[2 * smp + 1] = ei;
          } else {
            a.eloc[smp] = er;
          }
        }
      }
    }
  }
  for (int i = lane; i < N; i += 64) a.chain_sigma[int64_t(chain) * N + i] = sig[i];
  if (lane == 0 && a.n_acc) a.n_acc[chain] = acc_count;
  if (pt && lane == 0) {
    a.temp[chain] = ptT[wid];
    if (wid == 0 && a.n_swap) a.n_swap[chain / a.n_rep] = n_swaps;
  }
}

template <typename T, bool C, int R, bool TL, bool SM>
__global__ __launch_bounds__(256) void k_sweep(DevModel dm, Tables<T> tb, SweepArgs a) {
  sweep_block<T, C, R, TL, SM, (R <= 4)>(dm, tb, a, blockIdx.x * (blockDim.x >> 6));
}

// ---------------------------------------------------------------------------------
// Metropolis sweeps of wide models (float forms, more than 256 hidden units): the hidden
// units of one chain are split over the G wavefronts of a block, 64 KW units per
// wavefront (lane l of wavefront w owns units 64 (KW w + r) + l, r < KW), so that each
// wavefront holds few angles and rows and several blocks share a compute unit. Every
// wavefront draws the same random numbers and keeps its own copy of the spins. A proposal:
// each wavefront forms the ratio terms of its units and the float logarithm of their
// product in groups of four units per lane, sums it over its lanes (DPP) and writes the sum
// to LDS; after one barrier every wavefront adds the G sums in wavefront order and takes
// the same decision (slots alternate between consecutive non-identity proposals, so one
// barrier per proposal suffices). Theta is cached in double, t = tanh theta in float,
// updated as in k_sweep and recomputed from theta after every sweep. The C/S/W rows of a
// move are read from the parameter tables once the move is known not to be the identity.
// ---------------------------------------------------------------------------------
constexpr int kWideUnits = 8;   // hidden units per lane of one wavefront

// sum over the wavefront of x, valid in lane 63: DPP row sums, then the row broadcasts
__device__ __forceinline__ float wave_sum_to_last(float x) {
  x += dpp_v<DPP_QP_XOR1>(x);
  x += dpp_v<DPP_QP_XOR2>(x);
  x += dpp_v<DPP_ROR4>(x);
  x += dpp_v<DPP_ROR8>(x);
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), DPP_BCAST15, 0xA, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), DPP_BCAST31, 0xC, 0xF, false));
  return x;
}

// Hidden angles theta[c][j] = b_j + sum_i W_ji sigma_ci of every chain in double on the
// FP64 matrix cores (16x16x4): a wavefront takes 16 chains x 64 hidden units (four 16-unit
// tiles), the spins (+/-1) and the float weights are exact in double, so only the order of
// the double additions differs from a sequential sum. The four wavefronts of a block share
// the 64 hidden units: their weights are staged in LDS 64 sites at a time (one read of the
// table per block instead of per wavefront). Grid (ceil(C / 64), ceil(M / 64)).
constexpr int kTh64Sites = 64;

template <bool C>
__global__ __launch_bounds__(256) void k_theta64(int N, int M, int n_chains,
                                                 const int8_t *__restrict__ sigma,
                                                 const float *__restrict__ Wt,
                                                 const float *__restrict__ bv, double *theta) {
  typedef double doublex4_t __attribute__((ext_vector_type(4)));
  // [site of the chunk][hidden unit of the block] (re, im), zero past N and past M
  __shared__ float2 lw[kTh64Sites][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int c0 = blockIdx.x * 64 + wid * 16;
  const int jb = blockIdx.y * 64;
  const int crow = c0 + lo;
  const int8_t *srow = sigma + int64_t(crow < n_chains ? crow : 0) * N;
  doublex4_t ar[4], ai[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ar[q] = doublex4_t{0, 0, 0, 0};
    ai[q] = doublex4_t{0, 0, 0, 0};
  }
  for (int kc = 0; kc < N; kc += kTh64Sites) {
    if (kc > 0) __syncthreads();  // the previous chunk is no longer read
    for (int e = threadIdx.x; e < kTh64Sites * 64; e += 256) {
      const int kk = e >> 6, jj = e & 63;
      const int k = kc + kk, j = jb + jj;
      float2 w = make_float2(0.f, 0.f);
      if (k < N && j < M) {
        const int64_t x = int64_t(k) * M + j;
        w = C ? make_float2(Wt[2 * x], Wt[2 * x + 1]) : make_float2(Wt[x], 0.f);
      }
      lw[kk][jj] = w;
    }
    __syncthreads();
    const int kn = N - kc < kTh64Sites ? N - kc : kTh64Sites;
    for (int k0 = 0; k0 < kn; k0 += 4) {
      const int kk = k0 + hi, k = kc + kk;
      const double a = (crow < n_chains && kk < kn) ? double(srow[k]) : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float2 w = lw[kk < kTh64Sites ? kk : 0][16 * q + lo];
        ar[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, double(w.x), ar[q], 0, 0, 0);
        if constexpr (C)
          ai[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, double(w.y), ai[q], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = jb + 16 * q + lo;
    if (j >= M) continue;
    const double br = C ? double(bv[2 * j]) : double(bv[j]);
    const double bi = C ? double(bv[2 * j + 1]) : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = c0 + hi + 4 * r;
      if (c >= n_chains) continue;
      if (C) {
        theta[2 * (int64_t(c) * M + j)] = ar[q][r] + br;
        theta[2 * (int64_t(c) * M + j) + 1] = ai[q][r] + bi;
      } else {
        theta[int64_t(c) * M + j] = ar[q][r] + br;
      }
    }
  }
}

template <bool C>
__global__ __launch_bounds__(256, 3) void k_sweep_wide(DevModel dm, Tables<float> tb, SweepArgs a,
                                                    int G, const double *__restrict__ theta0) {
  typedef float T;
  constexpr int KW = kWideUnits;
  extern __shared__ __align__(16) unsigned char lds_u8[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int chain = blockIdx.x;
  const int N = dm.N, M = dm.M;
  const bool flip = dm.move == NQS_MOVE_FLIP;
  const T *gC = flip ? tb.fC : tb.bC;
  const T *gS = flip ? tb.fS : tb.bS;
  const T *gW = flip ? tb.Wt : tb.Wd;
  // LDS: spins of every wavefront [G][Npad], the two slot rows of wavefront sums [2][G],
  // then |visible-bias factor|^2 [2][rows] and the color-0 bonds [B0][2]
  int8_t *sig = reinterpret_cast<int8_t *>(lds_u8 + int64_t(wid) * a.Npad);
  float *slots = reinterpret_cast<float *>(lds_u8 + int64_t(G) * a.Npad);
  const int afn = flip ? N : dm.Btot;
  const int64_t aux_off = (int64_t(G) * a.Npad + 8 * G + 15) & ~int64_t(15);
  double *la2 = reinterpret_cast<double *>(lds_u8 + aux_off);
  int *lbond = reinterpret_cast<int *>(la2 + 2 * afn);
  {
    const double *afb = flip ? tb.fa : tb.ba;
    for (int e = threadIdx.x; e < 2 * afn; e += blockDim.x)
      la2[e] = afb[2 * e] * afb[2 * e] + afb[2 * e + 1] * afb[2 * e + 1];
    if (!flip)
      for (int e = threadIdx.x; e < 2 * dm.B0; e += blockDim.x) lbond[e] = dm.bonds[e];
  }
  for (int i = lane; i < N; i += 64) sig[i] = a.chain_sigma[int64_t(chain) * N + i];
  __syncthreads();

  // this lane's units, their angles in double and t = tanh(theta) in float
  const int j0 = 64 * KW * wid + lane;
  double thr[KW], thi[KW];
  V<T, C> t[KW];
#pragma unroll
  for (int r = 0; r < KW; ++r) {
    const int j = j0 + 64 * r;
    thr[r] = 0.0;
    thi[r] = 0.0;
    t[r] = vmake<T, C>(T(0), T(0));
    if (j < M) {
      V<double, C> acc;
      if (theta0) {
        acc = vload<double, C>(theta0, int64_t(chain) * M + j);
      } else {
        acc = vload<double, C>(tb.bv, j);
        for (int i = 0; i < N; ++i) {
          const double sv = double(sig[i]);
          V<double, C> w = vload<double, C>(tb.Wt, int64_t(i) * M + j);
          acc.re += sv * w.re;
          if (C) acc.im += sv * w.im;
        }
      }
      thr[r] = acc.re;
      thi[r] = C ? acc.im : 0.0;
      t[r] = vtanh<T, C>(vmake<T, C>(T(thr[r]), T(thi[r])));
    }
  }
  const uint32_t cid = a.chain_offset + uint32_t(chain);
  const int total = a.n_discard + a.n_sweeps;
  const bool sregs = N <= 256;
  int sp0 = 0, sp1 = 0, sp2 = 0, sp3 = 0;
  if (sregs) {
    sp0 = lane < N ? sig[lane] : 0;
    sp1 = lane + 64 < N ? sig[lane + 64] : 0;
    sp2 = lane + 128 < N ? sig[lane + 128] : 0;
    sp3 = lane + 192 < N ? sig[lane + 192] : 0;
  }
  int64_t acc_count = 0;
  int parity = 0;
  for (int sw = 0; sw < total; ++sw) {
    for (int st0 = 0; st0 < N; st0 += 64) {
      const int nst = N - st0 < 64 ? N - st0 : 64;
      int rowv = 0, iv = 0, kv = 0;
      float thp = 0.f, thm = 0.f;
      if (lane < nst) {
        const Philox4 w = philox4x32_10(cid, a.counter + uint32_t(sw), uint32_t(st0 + lane),
                                        TAG_PROPOSAL, a.k0, a.k1);
        if (flip) {
          iv = rng_index(w.w[0], uint32_t(N));
          rowv = iv;
          kv = iv;
        } else {
          rowv = rng_index(w.w[0], uint32_t(dm.B0));
          iv = lbond[2 * rowv];
          kv = lbond[2 * rowv + 1];
        }
        const double uv = rng_uniform(w.w[1], w.w[2]);
        const float lu = __log2f(float(uv));
        thp = lu - __log2f(float(la2[rowv]));
        thm = lu - __log2f(float(la2[afn + rowv]));
      }
      for (int l = 0; l < nst; ++l) {
        const int ic = __builtin_amdgcn_readlane(iv, l);
        const int kc = __builtin_amdgcn_readlane(kv, l);
        int s, sk;
        if (sregs) {
          s = __builtin_amdgcn_readlane(ic < 64 ? sp0 : (ic < 128 ? sp1 : (ic < 192 ? sp2 : sp3)),
                                        ic & 63);
          sk = flip ? -s
                    : __builtin_amdgcn_readlane(
                          kc < 64 ? sp0 : (kc < 128 ? sp1 : (kc < 192 ? sp2 : sp3)), kc & 63);
        } else {
          s = __builtin_amdgcn_readfirstlane(int(sig[ic]));
          sk = flip ? -s : __builtin_amdgcn_readfirstlane(int(sig[kc]));
        }
        if (sk == s) continue;  // an exchange of equal spins is the identity move
        const int row = __builtin_amdgcn_readlane(rowv, l);
        const T ts = T(s);
        V<T, C> cc[KW], ss[KW], term[KW];
#pragma unroll
        for (int r = 0; r < KW; ++r) {
          const int j = j0 + 64 * r < M ? j0 + 64 * r : 0;
          cc[r] = vload<T, C>(gC, int64_t(row) * M + j);
          ss[r] = vload<T, C>(gS, int64_t(row) * M + j);
        }
        float lp = 0.f;
#pragma unroll
        for (int r0 = 0; r0 < KW; r0 += 4) {
          float pm = 1.f;
#pragma unroll
          for (int r = r0; r < r0 + 4; ++r) {
            term[r] = vsub(cc[r], vscale(vmul(t[r], ss[r]), ts));
            if (j0 + 64 * r < M) pm *= float(vabs2(term[r]));
          }
          lp += __log2f(pm);
        }
        const float wsum = wave_sum_to_last(lp);
        if (lane == 63) slots[parity * G + wid] = wsum;
        __syncthreads();
        float tot = 0.f;
        for (int g = 0; g < G; ++g) tot += slots[parity * G + g];
        parity ^= 1;
        const float th = readlane_v(s > 0 ? thp : thm, l);
        const int accept = __builtin_amdgcn_readfirstlane(int(tot > th));
        if (accept) {
          // the angle change (W row of the move) is read only for accepted moves
          V<T, C> ww[KW];
#pragma unroll
          for (int r = 0; r < KW; ++r)
            ww[r] = vload<T, C>(gW, int64_t(row) * M + (j0 + 64 * r < M ? j0 + 64 * r : 0));
#pragma unroll
          for (int r = 0; r < KW; ++r) {
            if (j0 + 64 * r < M) {
              thr[r] -= 2.0 * double(s) * double(ww[r].re);
              if (C) thi[r] -= 2.0 * double(s) * double(ww[r].im);
              t[r] = vdiv(vsub(vmul(cc[r], t[r]), vscale(ss[r], ts)), term[r]);
            }
          }
          if (sregs) {
            if (ic < 64)
              sp0 = lane == (ic & 63) ? -s : sp0;
            else if (ic < 128)
              sp1 = lane == (ic & 63) ? -s : sp1;
            else if (ic < 192)
              sp2 = lane == (ic & 63) ? -s : sp2;
            else
              sp3 = lane == (ic & 63) ? -s : sp3;
            if (!flip) {
              if (kc < 64)
                sp0 = lane == (kc & 63) ? s : sp0;
              else if (kc < 128)
                sp1 = lane == (kc & 63) ? s : sp1;
              else if (kc < 192)
                sp2 = lane == (kc & 63) ? s : sp2;
              else
                sp3 = lane == (kc & 63) ? s : sp3;
            }
          }
          if (lane == 0) {
            sig[ic] = int8_t(-s);
            if (!flip) sig[kc] = int8_t(s);
          }
          if (!sregs) wave_sync();
          ++acc_count;
        }
      }
    }
    wave_sync();
    // end of sweep: tanh from the exact angles
#pragma unroll
    for (int r = 0; r < KW; ++r)
      if (j0 + 64 * r < M) t[r] = vtanh<T, C>(vmake<T, C>(T(thr[r]), T(thi[r])));
    if (wid == 0 && sw >= a.n_discard) {
      const int64_t smp = int64_t(sw - a.n_discard) * a.n_chains + chain;
      int8_t *dst = a.samples + smp * N;
      for (int i = lane; i < N; i += 64) dst[i] = sig[i];
    }
  }
  if (wid == 0) {
    for (int i = lane; i < N; i += 64) a.chain_sigma[int64_t(chain) * N + i] = sig[i];
    if (lane == 0 && a.n_acc) a.n_acc[chain] = acc_count;
  }
}

// ---------------------------------------------------------------------------------
// Batches of independent models in one launch: each block reads its job (one model's
// tables and arguments) and its first chain (or element block) from a block map built
// on the host, then runs the single-model body. Tables are read from global memory.
// ---------------------------------------------------------------------------------
template <typename T>
struct SweepJob {
  DevModel dm;
  Tables<T> tb;
  SweepArgs a;
};

// The sweep base of the counter is an argument, or read from device memory (counter_dev,
// advanced after the launch by k_advance_counter), so that the job table does not change
// from call to call and replays of a captured call continue the random stream.
template <typename T, bool C, int R>
__global__ __launch_bounds__(256) void k_sweep_batch(const SweepJob<T> *__restrict__ jobs,
                                                     const int2 *__restrict__ bmap,
                                                     uint32_t counter,
                                                     const uint64_t *counter_dev) {
  const int2 bm = bmap[blockIdx.x];  // (job, first chain of the block)
  SweepJob<T> J = jobs[bm.x];
  J.a.counter = counter_dev ? uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(*counter_dev)))
                            : counter;
  sweep_block<T, C, R, false, false>(J.dm, J.tb, J.a, bm.y);
}

__global__ void k_advance_counter(uint64_t *counter_dev, uint64_t by) {
  if (threadIdx.x == 0) *counter_dev += by;
}

template <typename T, typename PT>
struct TabJob {
  DevModel dm;
  Tables<T> tb;
  const PT *p;
  int quant, need_flip, need_bond, blocks;
};

template <typename T, bool C, typename PT>
__global__ void k_tables_batch(const TabJob<T, PT> *__restrict__ jobs,
                               const int2 *__restrict__ bmap) {
  const int2 bm = bmap[blockIdx.x];  // (job, block within the job)
  const TabJob<T, PT> J = jobs[bm.x];
  tables_body<T, C, PT>(J.dm, J.tb, J.p, J.quant, J.need_flip, J.need_bond, bm.y, J.blocks);
}

// ---------------------------------------------------------------------------------
// Local energy of arbitrary configurations from precomputed rows T[s][j] = tanh(theta_j)
// (the matrix-core kernel k_theta_tanh): one sample per wavefront, eight wavefronts per
// block sharing the C/S rows of the connected configurations, staged in LDS when they fit
// (TL). TP > 0 (M <= 16 TP <= 256): four configurations per pass, TP hidden tiles of 16
// per lane group (eloc_grouped); TP = 0: R hidden units per lane (eloc_regs).
// ---------------------------------------------------------------------------------
constexpr int kElocWaves = 8;
template <typename T, bool C, int R, bool TL, int TP>
__global__ __launch_bounds__(64 * kElocWaves) void k_local_energy(DevModel dm, Tables<T> tb,
                                                       const int8_t *__restrict__ sigma,
                                                       const T *__restrict__ Tm, int64_t n,
                                                       double *eloc, int Npad, int cs_rows) {
  extern __shared__ __align__(16) unsigned char lds_u8[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int N = dm.N, M = dm.M;
  constexpr int cs = C ? 2 : 1;
  T *lC = reinterpret_cast<T *>(lds_u8);
  T *lS = lC + int64_t(cs_rows) * M * cs;
  const int64_t tab_bytes = TL ? int64_t(2) * cs_rows * M * cs * int64_t(sizeof(T)) : 0;
  if constexpr (TL) {
    const T *gCe = dm.ham == NQS_TFIM ? tb.fC : tb.bC;
    const T *gSe = dm.ham == NQS_TFIM ? tb.fS : tb.bS;
    const int64_t ce = int64_t(cs_rows) * M * cs;
    for (int64_t e = threadIdx.x; e < ce; e += blockDim.x) {
      lC[e] = gCe[e];
      lS[e] = gSe[e];
    }
    __syncthreads();
  }
  int8_t *sig = reinterpret_cast<int8_t *>(lds_u8 + tab_bytes + int64_t(wid) * Npad);
  // persistent blocks: the staged rows serve every sample the block visits
  for (int64_t smp = int64_t(blockIdx.x) * (blockDim.x >> 6) + wid; smp < n;
       smp += int64_t(gridDim.x) * (blockDim.x >> 6)) {
    wave_sync();
    for (int i = lane; i < N; i += 64) sig[i] = sigma[smp * N + i];
    wave_sync();
    const T *trow = Tm + smp * M * cs;
    double er, ei;
    if constexpr (TP > 0) {
      eloc_grouped<T, C, TL, TP>(dm, tb, sig, trow, lane, lC, lS, er, ei);
    } else {
      V<T, C> t[R];
#pragma unroll
      for (int r = 0; r < R; ++r)
        t[r] = lane + 64 * r < M ? vload<T, C>(trow, lane + 64 * r) : vmake<T, C>(T(0), T(0));
      eloc_regs<T, C, R, TL>(dm, tb, sig, t, lane, lC, lS, er, ei);
    }
    if (lane == 0) {
      if (C) {
        eloc[2 * smp] = er;
        eloc[2 * smp + 1] = ei;
      } else {
        eloc[smp] = er;
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// Local energy for wide models (M > 256) whose tables do not fit in LDS: a block of
// kRowsWaves wavefronts takes one sample each (its tanh row in registers, R values per
// lane) and walks the candidate rows (sites for TFIM, bonds for Heisenberg) in chunks of
// KB rows. Each chunk's C/S rows are staged in LDS once and read by every wavefront whose
// sample connects them, so a block reads the tables once for its samples instead of once
// per sample. Same terms and product order as eloc_regs (Eq. 5).
// ---------------------------------------------------------------------------------
constexpr int kRowsWaves = 16;

template <typename T, bool C, int R>
__global__ __launch_bounds__(64 * kRowsWaves) void k_eloc_rows(DevModel dm, Tables<T> tb,
                                                               const int8_t *__restrict__ sigma,
                                                               const T *__restrict__ Tm,
                                                               int64_t n, double *eloc, int Npad,
                                                               int KB) {
  extern __shared__ __align__(16) unsigned char lds_u8[];
  constexpr int cs = C ? 2 : 1;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int N = dm.N, M = dm.M, B = dm.Btot;
  const bool tfim = dm.ham == NQS_TFIM;
  const int nrows = tfim ? (dm.h != 0.0 ? N : 0) : B;
  const T *gC = tfim ? tb.fC : tb.bC;
  const T *gS = tfim ? tb.fS : tb.bS;
  // [KB][Mp] values of the chunk's rows, Mp = 64 R: entries past M hold C = 1, S = 0, so
  // the product loop needs no bound test
  const int Mp = 64 * R;
  T *lC = reinterpret_cast<T *>(lds_u8);
  T *lS = lC + int64_t(KB) * Mp * cs;
  int8_t *sig = reinterpret_cast<int8_t *>(lS + int64_t(KB) * Mp * cs) + wid * Npad;
  const int64_t smp = int64_t(blockIdx.x) * kRowsWaves + wid;
  const bool ok = smp < n;
  const int64_t sr = ok ? smp : n - 1;
  for (int i = lane; i < N; i += 64) sig[i] = sigma[sr * N + i];
  V<T, C> t[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    t[r] = lane + 64 * r < M ? vload<T, C>(Tm + sr * M * cs, lane + 64 * r)
                             : vmake<T, C>(T(0), T(0));
  wave_sync();
  double diag = 0.0;
  for (int b = lane; b < B; b += 64)
    diag += dm.bond_diag[b] * double(sig[dm.bonds[2 * b]]) * double(sig[dm.bonds[2 * b + 1]]);
  double er = 0.0, ei = 0.0;
  for (int c0 = 0; c0 < nrows; c0 += KB) {
    const int kb = nrows - c0 < KB ? nrows - c0 : KB;
    __syncthreads();  // the previous chunk's rows are no longer read
    const int64_t ne = int64_t(kb) * Mp;
    for (int64_t e = threadIdx.x; e < ne; e += blockDim.x) {
      const int q = int(e / Mp), j = int(e - int64_t(q) * Mp);
      const int64_t g = int64_t(c0 + q) * M + j;
      vstore<T, C>(lC, e, j < M ? vload<T, C>(gC, g) : vmake<T, C>(T(1), T(0)));
      vstore<T, C>(lS, e, j < M ? vload<T, C>(gS, g) : vmake<T, C>(T(0), T(0)));
    }
    __syncthreads();
    if (!ok) continue;
    for (int q = 0; q < kb; ++q) {
      const int row = c0 + q;
      int s;
      bool conn;
      double el;
      if (tfim) {
        s = sig[row] > 0 ? 1 : -1;
        conn = true;
        el = -dm.h;
      } else {
        const int si = sig[dm.bonds[2 * row]], sk = sig[dm.bonds[2 * row + 1]];
        s = si > 0 ? 1 : -1;
        el = dm.bond_off[row];
        conn = si != sk && el != 0.0;
      }
      if (!__builtin_amdgcn_readfirstlane(int(conn))) continue;  // the same on every lane
      s = __builtin_amdgcn_readfirstlane(s);
      const T ts = T(s);
      V<T, C> p = vmake<T, C>(T(1), T(0));
      int pe = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int j = lane + 64 * r;
        const V<T, C> cc = vload<T, C>(lC, int64_t(q) * Mp + j);
        const V<T, C> ss = vload<T, C>(lS, int64_t(q) * Mp + j);
        p = vmul(p, vsub(cc, vscale(vmul(t[r], ss), ts)));
        if ((r & 3) == 3) vrenorm(p, pe);
      }
      vrenorm(p, pe);
      const V<T, C> w = wave_cprod_dpp(p, pe);
      const double *af = tfim ? tb.fa + 2 * (int64_t(s > 0 ? 0 : 1) * N + row)
                              : tb.ba + 2 * (int64_t(s > 0 ? 0 : 1) * B + row);
      const double rr = ldexp(double(w.re), pe), ri = C ? ldexp(double(w.im), pe) : 0.0;
      er += el * (rr * af[0] - ri * af[1]);
      ei += el * (rr * af[1] + ri * af[0]);
    }
  }
  const double dsum = wave_sum_dpp(diag);
  if (ok && lane == 0) {
    if (C) {
      eloc[2 * smp] = dsum + er;
      eloc[2 * smp + 1] = ei;
    } else {
      eloc[smp] = dsum + er;
    }
  }
}

// ---------------------------------------------------------------------------------
// Local energy with one sample per lane, for small models (M <= 16 TPM, N <= 64, at most
// 64 candidate rows, rows staged in LDS): the lane's tanh row sits in registers and the
// lane visits only the rows its sample connects (every site for TFIM, the bonds with
// opposite spins for Heisenberg), reading their C/S entries from LDS, and multiplies its
// own ratio terms, so no cross-lane reduction is needed; the loop runs as many passes as
// the lane with the most connected rows. In the last, partial grid-stride step several
// lanes share a sample and add their sums across lanes. Same terms as eloc_grouped (Eq. 5).
// ---------------------------------------------------------------------------------
template <typename T, bool C, int TPM>
__global__ __launch_bounds__(256) void k_eloc_lanes(DevModel dm, Tables<T> tb,
                                                     const int8_t *__restrict__ sigma,
                                                     const T *__restrict__ Tm, int64_t n,
                                                     double *eloc, int cs_rows) {
  extern __shared__ __align__(16) unsigned char lds_u8[];
  constexpr int cs = C ? 2 : 1;
  constexpr int MJ = 16 * TPM;
  const int N = dm.N, M = dm.M, B = dm.Btot;
  const bool tfim = dm.ham == NQS_TFIM;
  // tables staged transposed, [j][row] with a row stride of 64 (so lanes on different rows
  // read consecutive elements, at most two rows per bank pair, and element j sits at a
  // compile-time offset); entries past M hold C = 1, S = 0, so their ratio term is exactly
  // 1 and the product loop has no bound test. After the tables: the element of every row
  // and the visible-bias factors of either spin.
  constexpr int RS = 64;
  T *lC = reinterpret_cast<T *>(lds_u8);
  T *lS = lC + int64_t(MJ) * RS * cs;
  double *lel = reinterpret_cast<double *>(lS + int64_t(MJ) * RS * cs);  // [rows]
  double *laf = lel + cs_rows;  // [2][rows] complex
  {
    const T *gC = tfim ? tb.fC : tb.bC;
    const T *gS = tfim ? tb.fS : tb.bS;
    for (int e = threadIdx.x; e < cs_rows * MJ; e += blockDim.x) {
      const int r = e / MJ, j = e - r * MJ;
      V<T, C> cc = vmake<T, C>(T(1), T(0)), ss = vmake<T, C>(T(0), T(0));
      if (j < M) {
        cc = vload<T, C>(gC, int64_t(r) * M + j);
        ss = vload<T, C>(gS, int64_t(r) * M + j);
      }
      vstore<T, C>(lC, j * RS + r, cc);
      vstore<T, C>(lS, j * RS + r, ss);
    }
    const double *gaf = tfim ? tb.fa : tb.ba;
    for (int e = threadIdx.x; e < cs_rows; e += blockDim.x)
      lel[e] = tfim ? -dm.h : dm.bond_off[e];
    for (int e = threadIdx.x; e < 4 * cs_rows; e += blockDim.x) laf[e] = gaf[e];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nrows = tfim ? (dm.h != 0.0 ? N : 0) : B;
  // Whole grid-stride steps give every wavefront 64 samples, one per lane. The samples
  // left after them (fewer than 64 per wavefront) are spread over every wavefront: spw per wavefront,
  // L = 64 / spw lanes per sample, each lane taking every L-th of the sample's connected
  // rows; the L partial sums are then added across the lanes.
  const int64_t W = int64_t(gridDim.x) * (blockDim.x >> 6);
  const int64_t wg = int64_t(blockIdx.x) * (blockDim.x >> 6) + wid;
  const int64_t nfull = n / (64 * W) * (64 * W), rem = n - nfull;
  int spw = 1;
  while (int64_t(spw) * W < rem) spw <<= 1;
  const int64_t steps = nfull / (64 * W) + (rem > 0 ? 1 : 0);
  for (int64_t it = 0; it < steps; ++it) {
    const bool tail = it * 64 * W >= nfull;
    const int L = tail ? 64 / spw : 1;
    const int sub = lane & (L - 1);
    const int64_t base = tail ? nfull + wg * spw : it * 64 * W + wg * 64;
    if (base >= n) break;  // the same for every lane of the wavefront
    const int64_t smp = base + lane / L;
    const bool ok = smp < n;
    const int64_t sr = ok ? smp : n - 1;
    uint64_t mask = 0;  // bit i: spin i up
    const int8_t *row = sigma + sr * N;
    for (int i = 0; i < N; ++i) mask |= uint64_t(row[i] > 0) << i;
    V<T, C> t[MJ];
#pragma unroll
    for (int j = 0; j < MJ; ++j)
      t[j] = j < M ? vload<T, C>(Tm, sr * M + j) : vmake<T, C>(T(0), T(0));
    double diag = 0.0;
    for (int b = 0; b < B; ++b) {
      const int i = dm.bonds[2 * b], k = dm.bonds[2 * b + 1];
      const int si = ((mask >> i) & 1ull) ? 1 : -1, sk = ((mask >> k) & 1ull) ? 1 : -1;
      diag += dm.bond_diag[b] * double(si * sk);
    }
    // the rows this lane's sample connects (bit c of cmask) and the spin s of each (bit c
    // of upm: s = +1); each lane then visits only its own rows, in increasing order
    uint64_t cmask = 0, upm = 0;
    for (int c = 0; c < nrows; ++c) {
      bool conn, up;
      if (tfim) {
        up = (mask >> c) & 1ull;
        conn = true;
      } else {
        const int i = dm.bonds[2 * c], k = dm.bonds[2 * c + 1];
        const bool ui = (mask >> i) & 1ull, uk = (mask >> k) & 1ull;
        up = ui;
        conn = ui != uk && dm.bond_off[c] != 0.0;
      }
      cmask |= uint64_t(conn && ok) << c;
      upm |= uint64_t(up) << c;
    }
    if (L > 1) {
      // keep the connected rows whose rank among them is sub modulo L
      uint64_t keep = 0, rest = cmask;
      for (int rk = 0; rest != 0; ++rk) {
        const uint64_t bit = rest & (~rest + 1);
        if ((rk & (L - 1)) == sub) keep |= bit;
        rest ^= bit;
      }
      cmask = keep;
    }
    double er = 0.0, ei = 0.0;
    while (__ballot(cmask != 0)) {
      const bool have = cmask != 0;  // lanes without a row left take row 0 and discard it
      const int c = have ? int(__builtin_ctzll(cmask)) : 0;
      cmask &= cmask - 1;
      const int sgn = ((upm >> c) & 1ull) ? 1 : -1;
      const T ts = T(sgn);
      const T *crow = lC + c * cs, *srow = lS + c * cs;
      // four interleaved partial products (j mod 4), so that four independent
      // multiplication chains are in flight, then combined
      V<T, C> pq[4];
      int peq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pq[q] = vmake<T, C>(T(1), T(0));
        peq[q] = 0;
      }
#pragma unroll
      for (int j = 0; j < MJ; ++j) {
        const V<T, C> cc = vload<T, C>(crow, j * RS), ss = vload<T, C>(srow, j * RS);
        pq[j & 3] = vmul(pq[j & 3], vsub(cc, vscale(vmul(t[j], ss), ts)));
        if ((j & 31) >= 28) vrenorm(pq[j & 3], peq[j & 3]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) vrenorm(pq[q], peq[q]);
      V<T, C> p = vmul(vmul(pq[0], pq[1]), vmul(pq[2], pq[3]));
      int pe = (peq[0] + peq[1]) + (peq[2] + peq[3]);
      vrenorm(p, pe);
      const double *af = laf + 2 * (int64_t(sgn > 0 ? 0 : 1) * cs_rows + c);
      const double el = lel[c];
      const double rr = ldexp(double(p.re), pe), ri = C ? ldexp(double(p.im), pe) : 0.0;
      if (have) {
        er += el * (rr * af[0] - ri * af[1]);
        ei += el * (rr * af[1] + ri * af[0]);
      }
    }
    for (int o = L >> 1; o > 0; o >>= 1) {
      er += __shfl_xor(er, o);
      ei += __shfl_xor(ei, o);
    }
    if (ok && sub == 0) {
      if (C) {
        eloc[2 * smp] = diag + er;
        eloc[2 * smp + 1] = ei;
      } else {
        eloc[smp] = diag + er;
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// log psi. One sample per wavefront; theta, ln cosh and the sums in double for every
// compute precision (near the complex zeros of cosh theta, rounding theta to FP32 alone
// would dominate the error; log psi is not on the sampling or SR path).
// ---------------------------------------------------------------------------------
template <typename T, bool C>
__global__ __launch_bounds__(256) void k_log_psi(DevModel dm, Tables<T> tb,
                                                  const int8_t *__restrict__ sigma, int64_t n,
                                                  double *out, int Npad) {
  extern __shared__ int8_t lds_s8[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t smp = int64_t(blockIdx.x) * (blockDim.x >> 6) + wid;
  if (smp >= n) return;
  const int N = dm.N, M = dm.M;
  int8_t *sig = lds_s8 + wid * Npad;
  for (int i = lane; i < N; i += 64) sig[i] = sigma[smp * N + i];
  wave_sync();
  double lr = 0.0, li = 0.0;
  for (int j = lane; j < M; j += 64) {
    V<double, C> acc = vload<double, C>(tb.bv, j);
    for (int i = 0; i < N; ++i) {
      double s = double(sig[i]);
      V<double, C> w = vload<double, C>(tb.Wt, int64_t(i) * M + j);
      acc.re += s * w.re;
      if (C) acc.im += s * w.im;
    }
    V<double, C> lc = vlncosh<double, C>(acc);
    lr += lc.re;
    if (C) li += lc.im;
  }
  for (int i = lane; i < N; i += 64) {
    lr += tb.av[2 * i] * double(sig[i]);
    li += tb.av[2 * i + 1] * double(sig[i]);
  }
  lr = wave_sum(lr);
  li = wave_sum(li);
  if (lane == 0) {
    if (C) {
      out[2 * smp] = lr;
      out[2 * smp + 1] = li;
    } else {
      out[smp] = lr;
    }
  }
}

// Job structs are compared byte by byte with the previous upload of their table (a table
// is uploaded again only when it changed), so every struct that goes into one starts
// zero-filled: padding bytes are then the same from call to call.
template <typename S>
inline void zero_fill(S &x) {
  static_assert(std::is_trivially_copyable<S>::value, "job structs are plain data");
  memset(static_cast<void *>(&x), 0, sizeof(S));
}

template <typename T>
Tables<T> tables_of(const nqs_model *m) {
  Tables<T> tb;
  zero_fill(tb);
  tb.Wt = (T *)m->tab_ptrs[0];
  tb.bv = (T *)m->tab_ptrs[1];
  tb.fC = (T *)m->tab_ptrs[2];
  tb.fS = (T *)m->tab_ptrs[3];
  tb.bC = (T *)m->tab_ptrs[4];
  tb.bS = (T *)m->tab_ptrs[5];
  tb.fa = (double *)m->tab_ptrs[10];
  tb.ba = (double *)m->tab_ptrs[11];
  tb.av = (double *)m->tab_ptrs[12];
  tb.Wd = (T *)m->tab_ptrs[13];
  return tb;
}

inline int round_up(int x, int a) { return (x + a - 1) / a * a; }

template <typename T, bool C>
hipError_t tables_t(const nqs_model *m, const void *params, hipStream_t st) {
  DevModel dm = dev_model(m);
  Tables<T> tb = tables_of<T>(m);
  int64_t total = int64_t(m->N) * m->M + int64_t(m->Btot) * m->M + m->M + m->N + m->Btot;
  int blocks = int((total + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  int quant = m->prec == NQS_BF16;
  if (m->prec == NQS_F64)
    hipLaunchKernelGGL((k_tables<T, C, double>), dim3(blocks), dim3(256), 0, st, dm, tb,
                       (const double *)params, quant, int(m->need_flip), int(m->need_bond));
  else
    hipLaunchKernelGGL((k_tables<T, C, float>), dim3(blocks), dim3(256), 0, st, dm, tb,
                       (const float *)params, quant, int(m->need_flip), int(m->need_bond));
  return hipGetLastError();
}

// LDS of the sweep after the wavefronts' regions: |visible-bias factor|^2 of every row for
// either spin (2 x rows doubles) and, for exchange moves, the color-0 bonds (2 x B0 ints)
inline size_t sweep_aux_lds(const nqs_model *m) {
  const bool flip = m->move == NQS_MOVE_FLIP;
  const int afn = flip ? m->N : m->Btot;
  return size_t(16) * afn + (flip ? size_t(0) : size_t(8) * m->B[0]);
}

template <typename T, bool C, int R>
hipError_t sweep_r(const nqs_model *m, int8_t *cs, int n_chains, int n_sweeps, int n_discard,
                   uint64_t seed, uint64_t counter, int chain_offset, int8_t *samples,
                   int64_t *n_acc, void *eloc, void *scratch, hipStream_t st,
                   const PtArgs *pt) {
  // tempering: one block per tempered chain, one wavefront per replica
  const int wpb = pt ? pt->n_rep : 4;
  SweepArgs a;
  memset(static_cast<void *>(&a), 0, sizeof a);
  if (pt) {
    if (pt->n_rep < 2 || pt->n_rep > kMaxReplicas || n_chains % pt->n_rep) return hipErrorInvalidValue;
    a.n_rep = pt->n_rep;
    a.temp = pt->temp;
    a.n_swap = pt->n_swap;
    a.group_offset = uint32_t(chain_offset);
    for (int r = 0; r < pt->n_rep; ++r) a.betas[r] = 1.0 - double(r) / double(pt->n_rep);
    chain_offset *= pt->n_rep;   // proposal streams: (chain_offset + c) R + w
  }
  a.chain_sigma = cs;
  a.n_chains = n_chains;
  a.n_sweeps = n_sweeps;
  a.n_discard = n_discard;
  a.k0 = uint32_t(seed & 0xffffffffu);
  a.k1 = uint32_t(seed >> 32);
  a.counter = uint32_t(counter);
  a.chain_offset = uint32_t(chain_offset);
  a.samples = samples;
  a.n_acc = n_acc;
  a.eloc = (double *)eloc;
  const bool flip = m->move == NQS_MOVE_FLIP;
  a.cs_rows = m->ham == NQS_TFIM ? m->N : m->Btot;
  a.w_rows = flip ? m->N : m->B[0];
  a.Npad = round_up(m->N, 16);
  a.wave_bytes = a.Npad + round_up(m->M * int(sizeof(V<T, C>)), 16);
  const size_t wave_lds = size_t(wpb) * a.wave_bytes;
  const size_t tab_lds =
      size_t(2 * a.cs_rows + a.w_rows) * m->M * sizeof(T) * (C ? 2 : 1);
  // the visible-bias factors and bonds after the wavefronts' regions (16-byte aligned), and
  // with tempering the replicas' log amplitudes and temperature indices
  const size_t aux = sweep_aux_lds(m) + (pt ? 16 + 12 * kMaxReplicas : 0);
  auto with_aux = [&](size_t base) { return (base + 15) / 16 * 16 + aux; };
  // the staged C/S rows serve both the moves and the local energy only when the move
  // set is contained in the connected set: flips with TFIM, exchanges with Heisenberg
  const bool shared_rows = (m->ham == NQS_TFIM && flip) || (m->ham == NQS_HEISENBERG && !flip);
  dim3 grid((n_chains + wpb - 1) / wpb);
  const bool tl = shared_rows && with_aux(tab_lds + wave_lds) <= size_t(m->max_lds);
  if constexpr (R <= 4) {
    time_begin(m, NQS_TIME_SWEEP);
    time_mark(m, NQS_TIME_SWEEP, 0, st);
    if (m->N <= 64) {
      if (tl)
        hipLaunchKernelGGL((k_sweep<T, C, R, true, true>), grid, dim3(64 * wpb),
                           with_aux(tab_lds + wave_lds), st, dev_model(m), tables_of<T>(m), a);
      else
        hipLaunchKernelGGL((k_sweep<T, C, R, false, true>), grid, dim3(64 * wpb),
                           with_aux(wave_lds), st, dev_model(m), tables_of<T>(m), a);
      time_mark(m, NQS_TIME_SWEEP, 1, st);
      return hipGetLastError();
    }
  }
  if constexpr (sizeof(T) == 4 && R > 4) {
    if (!tl) {
      if (pt) return hipErrorNotSupported;   // the wide sweep does not temper
      // wide models: the chains' angles on the matrix cores (into the model's scratch, when
      // given), then the hidden units of a chain split over G wavefronts of one block
      const double *th0 = nullptr;
      if (scratch) {
        hipLaunchKernelGGL((k_theta64<C>), dim3((n_chains + 63) / 64, (m->M + 63) / 64),
                           dim3(256), 0, st, m->N, m->M, n_chains, (const int8_t *)cs,
                           (const float *)m->tab_ptrs[0], (const float *)m->tab_ptrs[1],
                           (double *)scratch);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        th0 = (const double *)scratch;
      }
      const int G = (m->M + 64 * kWideUnits - 1) / (64 * kWideUnits);
      const size_t lds = ((size_t(G) * a.Npad + 8 * G + 15) / 16 * 16) + aux;
      time_begin(m, NQS_TIME_SWEEP);
      time_mark(m, NQS_TIME_SWEEP, 0, st);
      hipLaunchKernelGGL((k_sweep_wide<C>), dim3(n_chains), dim3(64 * G), lds, st,
                         dev_model(m), tables_of<float>(m), a, G, th0);
      time_mark(m, NQS_TIME_SWEEP, 1, st);
      return hipGetLastError();
    }
  }
  if constexpr (R > 4) {
    time_begin(m, NQS_TIME_SWEEP);
    time_mark(m, NQS_TIME_SWEEP, 0, st);
  }
  if (tl) {
    hipLaunchKernelGGL((k_sweep<T, C, R, true, false>), grid, dim3(64 * wpb),
                       with_aux(tab_lds + wave_lds), st, dev_model(m), tables_of<T>(m), a);
  } else {
    hipLaunchKernelGGL((k_sweep<T, C, R, false, false>), grid, dim3(64 * wpb),
                       with_aux(wave_lds), st, dev_model(m), tables_of<T>(m), a);
  }
  time_mark(m, NQS_TIME_SWEEP, 1, st);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t sweep_t(const nqs_model *m, int8_t *cs, int n_chains, int n_sweeps, int n_discard,
                   uint64_t seed, uint64_t counter, int chain_offset, int8_t *samples,
                   int64_t *n_acc, void *eloc, void *scratch, hipStream_t st,
                   const PtArgs *pt) {
  int r = (m->M + 63) / 64;
#define NQS_SWEEP_CASE(RR)                                                                 \
  if (r <= RR)                                                                             \
    return sweep_r<T, C, RR>(m, cs, n_chains, n_sweeps, n_discard, seed, counter,          \
                             chain_offset, samples, n_acc, eloc, scratch, st, pt);
  NQS_SWEEP_CASE(1)
  NQS_SWEEP_CASE(2)
  NQS_SWEEP_CASE(4)
  NQS_SWEEP_CASE(8)
  NQS_SWEEP_CASE(16)
  NQS_SWEEP_CASE(32)
#undef NQS_SWEEP_CASE
  return hipErrorInvalidValue;
}

template <typename T, bool C, int R, int TP>
hipError_t eloc_r(const nqs_model *m, const int8_t *sigma, const void *Tm, int64_t n,
                  void *eloc, hipStream_t st) {
  const int Npad = round_up(m->N, 16);
  const int wpb = kElocWaves;
  const int cs_rows = m->ham == NQS_TFIM ? m->N : m->Btot;
  const size_t tab_lds = size_t(2) * cs_rows * m->M * sizeof(T) * (C ? 2 : 1);
  const size_t wave_lds = size_t(wpb) * Npad;
  // persistent grid: as many blocks as fit on the device at once (at most 4 per CU)
  const bool tl = tab_lds + wave_lds <= size_t(m->max_lds) / 2;
  int per_cu = 4;
  if (tl) {
    const int by_lds = int(size_t(160 * 1024) / (tab_lds + wave_lds));
    per_cu = by_lds < 1 ? 1 : (by_lds < 4 ? by_lds : 4);
  }
  int64_t blocks = (n + wpb - 1) / wpb;
  if (blocks > int64_t(per_cu) * m->cu_count) blocks = int64_t(per_cu) * m->cu_count;
  dim3 grid((unsigned)blocks);
  if (tl)
    hipLaunchKernelGGL((k_local_energy<T, C, R, true, TP>), grid, dim3(64 * wpb),
                       tab_lds + wave_lds, st, dev_model(m), tables_of<T>(m), sigma,
                       (const T *)Tm, n, (double *)eloc, Npad, cs_rows);
  else
    hipLaunchKernelGGL((k_local_energy<T, C, R, false, TP>), grid, dim3(64 * wpb), wave_lds, st,
                       dev_model(m), tables_of<T>(m), sigma, (const T *)Tm, n, (double *)eloc,
                       Npad, cs_rows);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t eloc_t(const nqs_model *m, const int8_t *sigma, const void *Tm, int64_t n,
                  void *eloc, hipStream_t st) {
  if (n == 0) return hipSuccess;
  // M <= 256: the smallest tile count of 16 hidden units per lane group covering M
  const int tp = (m->M + 15) / 16;
  // small models: one sample per lane (FP64 complex rows beyond 48 hidden units would
  // exceed 256 registers per lane; those keep the grouped kernel)
  if (tp <= 6 && m->N <= 64 && (sizeof(T) == 4 || !C || tp <= 3)) {
    const int cs_rows = m->ham == NQS_TFIM ? m->N : m->Btot;
    // both tables transposed with a row stride of 64, then the row elements and the
    // visible-bias factors (doubles)
    const size_t tab_lds =
        size_t(2) * 64 * (16 * tp) * sizeof(T) * (C ? 2 : 1) + size_t(40) * cs_rows;
    if (cs_rows <= 64 && tab_lds <= size_t(m->max_lds) * 5 / 8) {
      // one block of four wavefronts per compute unit (the row in registers takes up to
      // 512 registers per lane)
      int64_t blocks = (n + 255) / 256;
      // up to 48 hidden units the row and products fit two wavefronts per SIMD, when two
      // blocks' tables also fit the LDS of a compute unit (the spreading of the last
      // grid-stride step assumes every block is resident at once)
      int per_cu = tp <= 3 ? 2 : 1;
      const int by_lds = int(size_t(m->max_lds) / tab_lds);
      if (per_cu > by_lds) per_cu = by_lds < 1 ? 1 : by_lds;
      if (blocks > int64_t(per_cu) * m->cu_count) blocks = int64_t(per_cu) * m->cu_count;
#define NQS_ELOC_LANES(TPM)                                                                   \
  if (tp <= TPM) {                                                                            \
    if (tab_lds > 65536) {                                                                    \
      const hipError_t e = hipFuncSetAttribute(                                               \
          reinterpret_cast<const void *>(k_eloc_lanes<T, C, TPM>),                            \
          hipFuncAttributeMaxDynamicSharedMemorySize, m->max_lds);                            \
      if (e != hipSuccess) return e;                                                          \
    }                                                                                         \
    hipLaunchKernelGGL((k_eloc_lanes<T, C, TPM>), dim3(unsigned(blocks)), dim3(256), tab_lds, \
                       st, dev_model(m), tables_of<T>(m), sigma, (const T *)Tm, n,            \
                       (double *)eloc, cs_rows);                                              \
    return hipGetLastError();                                                                 \
  }
      NQS_ELOC_LANES(1) NQS_ELOC_LANES(2) NQS_ELOC_LANES(3)
      NQS_ELOC_LANES(4) NQS_ELOC_LANES(5) NQS_ELOC_LANES(6)
#undef NQS_ELOC_LANES
    }
  }
  if (tp <= 2) return eloc_r<T, C, 1, 2>(m, sigma, Tm, n, eloc, st);
  if (tp <= 3) return eloc_r<T, C, 1, 3>(m, sigma, Tm, n, eloc, st);
  if (tp <= 4) return eloc_r<T, C, 1, 4>(m, sigma, Tm, n, eloc, st);
  if (tp <= 5) return eloc_r<T, C, 1, 5>(m, sigma, Tm, n, eloc, st);
  if (tp <= 6) return eloc_r<T, C, 1, 6>(m, sigma, Tm, n, eloc, st);
  if (tp <= 8) return eloc_r<T, C, 1, 8>(m, sigma, Tm, n, eloc, st);
  if (tp <= 12) return eloc_r<T, C, 1, 12>(m, sigma, Tm, n, eloc, st);
  if (tp <= 16) return eloc_r<T, C, 1, 16>(m, sigma, Tm, n, eloc, st);
  const int r = (m->M + 63) / 64;
  {
    // wide models whose tables exceed LDS: chunks of rows staged per block of samples
    const int cs_rows = m->ham == NQS_TFIM ? m->N : m->Btot;
    const int Npad = round_up(m->N, 16);
    // rows padded to 64 R values, R the register count of the instance launched below
    const int Rsel = r <= 8 ? 8 : (r <= 16 ? 16 : 32);
    const size_t per_row = size_t(2) * 64 * Rsel * sizeof(T) * (C ? 2 : 1);
    const size_t tab_lds = size_t(2) * cs_rows * m->M * sizeof(T) * (C ? 2 : 1);
    const size_t fixed = size_t(kRowsWaves) * Npad;
    const int64_t fit = int64_t((size_t(m->max_lds) - fixed) / per_row);
    if (tab_lds > size_t(m->max_lds) / 2 && fit >= 1) {
      const int KB = int(fit < cs_rows ? fit : (cs_rows > 0 ? cs_rows : 1));
      const size_t lds = size_t(KB) * per_row + fixed;
      const dim3 grid(unsigned((n + kRowsWaves - 1) / kRowsWaves));
      auto go = [&](auto kern) -> hipError_t {
        // dynamic LDS beyond 64 KiB is opted into per instantiation
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 m->max_lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, grid, dim3(64 * kRowsWaves), lds, st, dev_model(m),
                           tables_of<T>(m), sigma, (const T *)Tm, n, (double *)eloc, Npad, KB);
        return hipGetLastError();
      };
      if (r <= 8) return go(k_eloc_rows<T, C, 8>);
      if (r <= 16) return go(k_eloc_rows<T, C, 16>);
      return go(k_eloc_rows<T, C, 32>);
    }
  }
  if (r <= 8) return eloc_r<T, C, 8, 0>(m, sigma, Tm, n, eloc, st);
  if (r <= 16) return eloc_r<T, C, 16, 0>(m, sigma, Tm, n, eloc, st);
  return eloc_r<T, C, 32, 0>(m, sigma, Tm, n, eloc, st);
}

template <typename T, bool C>
hipError_t logpsi_t(const nqs_model *m, const int8_t *sigma, int64_t n, void *out,
                    hipStream_t st) {
  if (n == 0) return hipSuccess;
  int Npad = round_up(m->N, 16);
  const int wpb = 4;
  dim3 grid(unsigned((n + wpb - 1) / wpb));
  hipLaunchKernelGGL((k_log_psi<T, C>), grid, dim3(64 * wpb), size_t(wpb) * Npad, st,
                     dev_model(m), tables_of<T>(m), sigma, n, (double *)out, Npad);
  return hipGetLastError();
}

}  // namespace

namespace {

template <typename T, bool C, int R>
hipError_t sample_batch_r(nqs_batch *b, const std::vector<BatchSampleItem> &items,
                          int n_sweeps, int n_discard, uint64_t counter, uint64_t *counter_dev,
                          hipStream_t st) {
  typedef typename std::conditional<std::is_same<T, double>::value, double, float>::type PT;
  const int wpb = 4;
  std::vector<TabJob<T, PT>> tj;
  std::vector<int2> tmap;
  std::vector<SweepJob<T>> sj;
  std::vector<int2> smap;
  size_t wave_max = 0, aux_max = 0;
  for (size_t k = 0; k < items.size(); ++k) {
    const BatchSampleItem &it = items[k];
    const nqs_model *m = it.m;
    TabJob<T, PT> t;
    zero_fill(t);
    t.dm = dev_model(m);
    t.tb = tables_of<T>(m);
    t.p = (const PT *)it.params;
    t.quant = m->prec == NQS_BF16;
    t.need_flip = int(m->need_flip);
    t.need_bond = int(m->need_bond);
    const int64_t total =
        int64_t(m->N) * m->M + int64_t(m->Btot) * m->M + m->M + m->N + m->Btot;
    t.blocks = int((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    for (int q = 0; q < t.blocks; ++q) tmap.push_back(make_int2(int(k), q));
    tj.push_back(t);
    SweepJob<T> w;
    zero_fill(w);
    w.dm = dev_model(m);
    w.tb = tables_of<T>(m);
    SweepArgs &a = w.a;
    a.chain_sigma = it.chains;
    a.n_chains = it.n_chains;
    a.n_sweeps = n_sweeps;
    a.n_discard = n_discard;
    a.k0 = uint32_t(it.seed & 0xffffffffu);
    a.k1 = uint32_t(it.seed >> 32);
    a.counter = 0;  // a launch argument (the table stays the same from call to call)
    a.chain_offset = 0;
    a.samples = it.samples;
    a.n_acc = it.n_acc;
    a.eloc = (double *)it.eloc;
    a.cs_rows = m->ham == NQS_TFIM ? m->N : m->Btot;
    a.w_rows = m->move == NQS_MOVE_FLIP ? m->N : m->B[0];
    a.Npad = round_up(m->N, 16);
    a.wave_bytes = a.Npad + round_up(m->M * int(sizeof(V<T, C>)), 16);
    if (size_t(a.wave_bytes) > wave_max) wave_max = size_t(a.wave_bytes);
    if (sweep_aux_lds(m) > aux_max) aux_max = sweep_aux_lds(m);
    for (int c = 0; c < it.n_chains; c += wpb) smap.push_back(make_int2(int(k), c));
    sj.push_back(w);
  }
  if (smap.empty()) return hipSuccess;
  hipError_t e;
  if ((e = b->tab_jobs.upload(tj.data(), tj.size() * sizeof(tj[0]), st)) != hipSuccess) return e;
  if ((e = b->tab_map.upload(tmap.data(), tmap.size() * sizeof(int2), st)) != hipSuccess) return e;
  if ((e = b->sweep_jobs.upload(sj.data(), sj.size() * sizeof(sj[0]), st)) != hipSuccess) return e;
  if ((e = b->sweep_map.upload(smap.data(), smap.size() * sizeof(int2), st)) != hipSuccess)
    return e;
  if (!b->tab_jobs.d || !b->tab_map.d || !b->sweep_jobs.d || !b->sweep_map.d)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_tables_batch<T, C, PT>), dim3(unsigned(tmap.size())), dim3(256), 0, st,
                     (const TabJob<T, PT> *)b->tab_jobs.d, (const int2 *)b->tab_map.d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((k_sweep_batch<T, C, R>), dim3(unsigned(smap.size())), dim3(64 * wpb),
                     (size_t(wpb) * wave_max + 15) / 16 * 16 + aux_max, st,
                     (const SweepJob<T> *)b->sweep_jobs.d, (const int2 *)b->sweep_map.d,
                     uint32_t(counter), (const uint64_t *)counter_dev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (counter_dev) {
    hipLaunchKernelGGL(k_advance_counter, dim3(1), dim3(64), 0, st, counter_dev,
                       uint64_t(n_discard) + uint64_t(n_sweeps));
    e = hipGetLastError();
  }
  return e;
}

template <typename T, bool C>
hipError_t sample_batch_t(nqs_batch *b, const std::vector<BatchSampleItem> &items,
                          int n_sweeps, int n_discard, uint64_t counter, uint64_t *counter_dev,
                          hipStream_t st) {
  int r = 1;
  for (const BatchSampleItem &it : items) {
    const int rk = (it.m->M + 63) / 64;
    if (rk > r) r = rk;
  }
  if (r <= 1) return sample_batch_r<T, C, 1>(b, items, n_sweeps, n_discard, counter, counter_dev, st);
  if (r <= 2) return sample_batch_r<T, C, 2>(b, items, n_sweeps, n_discard, counter, counter_dev, st);
  if (r <= 4) return sample_batch_r<T, C, 4>(b, items, n_sweeps, n_discard, counter, counter_dev, st);
  if (r <= 8) return sample_batch_r<T, C, 8>(b, items, n_sweeps, n_discard, counter, counter_dev, st);
  if (r <= 16) return sample_batch_r<T, C, 16>(b, items, n_sweeps, n_discard, counter, counter_dev, st);
  return sample_batch_r<T, C, 32>(b, items, n_sweeps, n_discard, counter, counter_dev, st);
}

template <typename T, bool C>
hipError_t tables_batch_t(nqs_batch *b, const std::vector<const void *> &params,
                          hipStream_t st) {
  typedef typename std::conditional<std::is_same<T, double>::value, double, float>::type PT;
  std::vector<TabJob<T, PT>> tj;
  std::vector<int2> tmap;
  for (size_t k = 0; k < params.size(); ++k) {
    const nqs_model *m = b->models[k];
    TabJob<T, PT> t;
    zero_fill(t);
    t.dm = dev_model(m);
    t.tb = tables_of<T>(m);
    t.p = (const PT *)params[k];
    t.quant = m->prec == NQS_BF16;
    t.need_flip = int(m->need_flip);
    t.need_bond = int(m->need_bond);
    const int64_t total =
        int64_t(m->N) * m->M + int64_t(m->Btot) * m->M + m->M + m->N + m->Btot;
    t.blocks = int((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    for (int q = 0; q < t.blocks; ++q) tmap.push_back(make_int2(int(k), q));
    tj.push_back(t);
  }
  hipError_t e;
  if ((e = b->tab_jobs.upload(tj.data(), tj.size() * sizeof(tj[0]), st)) != hipSuccess) return e;
  if ((e = b->tab_map.upload(tmap.data(), tmap.size() * sizeof(int2), st)) != hipSuccess) return e;
  if (!b->tab_jobs.d || !b->tab_map.d) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_tables_batch<T, C, PT>), dim3(unsigned(tmap.size())), dim3(256), 0, st,
                     (const TabJob<T, PT> *)b->tab_jobs.d, (const int2 *)b->tab_map.d);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tables_batch(nqs_batch *b, const std::vector<const void *> &params,
                               hipStream_t st) {
  if (params.empty()) return hipSuccess;
  const nqs_model *m = b->models[0];
  return use_double(m) ? (m->is_complex ? tables_batch_t<double, true>(b, params, st)
                                        : tables_batch_t<double, false>(b, params, st))
                       : (m->is_complex ? tables_batch_t<float, true>(b, params, st)
                                        : tables_batch_t<float, false>(b, params, st));
}

hipError_t launch_sample_batch(nqs_batch *b, const std::vector<BatchSampleItem> &items,
                               int n_sweeps, int n_discard, uint64_t counter,
                               uint64_t *counter_dev, hipStream_t st) {
  if (items.empty()) return hipSuccess;
  const nqs_model *m = items[0].m;
#define NQS_SB(T, C) sample_batch_t<T, C>(b, items, n_sweeps, n_discard, counter, counter_dev, st)
  return use_double(m) ? (m->is_complex ? NQS_SB(double, true) : NQS_SB(double, false))
                       : (m->is_complex ? NQS_SB(float, true) : NQS_SB(float, false));
#undef NQS_SB
}

#define NQS_DISPATCH(FN, ...)                                                              \
  (use_double(m) ? (m->is_complex ? FN<double, true>(__VA_ARGS__)                          \
                                  : FN<double, false>(__VA_ARGS__))                        \
                 : (m->is_complex ? FN<float, true>(__VA_ARGS__)                           \
                                  : FN<float, false>(__VA_ARGS__)))

hipError_t launch_tables(const nqs_model *m, const void *params, hipStream_t st) {
  return NQS_DISPATCH(tables_t, m, params, st);
}

hipError_t launch_chain_init(const nqs_model *m, int8_t *sig, int n_chains, uint64_t seed,
                             int chain_offset, hipStream_t st) {
  uint32_t k0 = uint32_t(seed & 0xffffffffu), k1 = uint32_t(seed >> 32);
  if (m->move == NQS_MOVE_FLIP) {
    int64_t total = int64_t(n_chains) * m->N;
    hipLaunchKernelGGL(k_init_flip, dim3(unsigned((total + 255) / 256)), dim3(256), 0, st, sig,
                       n_chains, m->N, k0, k1, uint32_t(chain_offset));
  } else {
    hipLaunchKernelGGL(k_init_sz0, dim3(unsigned((n_chains + 63) / 64)), dim3(64), 0, st, sig,
                       n_chains, m->N, k0, k1, uint32_t(chain_offset));
  }
  return hipGetLastError();
}

hipError_t launch_sweep(const nqs_model *m, int8_t *chain_sigma, int n_chains, int n_sweeps,
                        int n_discard, uint64_t seed, uint64_t counter, int chain_offset,
                        int8_t *samples, int64_t *n_acc, void *eloc, void *scratch,
                        hipStream_t st, const PtArgs *pt) {
  return NQS_DISPATCH(sweep_t, m, chain_sigma, n_chains, n_sweeps, n_discard, seed, counter,
                      chain_offset, samples, n_acc, pt ? nullptr : eloc, scratch, st, pt);
}

size_t sweep_scratch_bytes(const nqs_model *m, int n_chains) {
  // the wide sweep's angles [chains][M] in (complex) double; other shapes need none
  const bool wide = !use_double(m) && (m->M + 63) / 64 > 4;
  return wide ? size_t(n_chains) * m->M * (m->is_complex ? 16 : 8) : 0;
}

hipError_t launch_local_energy(const nqs_model *m, const int8_t *sigma, const void *Tm,
                               int64_t n, void *eloc, hipStream_t st) {
  return NQS_DISPATCH(eloc_t, m, sigma, Tm, n, eloc, st);
}

hipError_t launch_log_psi(const nqs_model *m, const int8_t *sigma, int64_t n, void *out,
                          hipStream_t st) {
  return NQS_DISPATCH(logpsi_t, m, sigma, n, out, st);
}
