/*
 * nqs.h - C ABI of libnqs, an MI355X (gfx950) implementation of the data-parallel hot
 * path of variational Monte Carlo with a restricted-Boltzmann-machine quantum state, as
 * described in the NetKet paper (Carleo et al., 2019), Sec. 2.2.
 *
 * Conventions for every entry point:
 *  - Pointers marked (device) are HIP device pointers owned by the caller; the library
 *    only borrows them for the duration of the call. Pointers marked (host) are host
 *    memory. The library allocates device memory only for the per-model tables created
 *    in nqs_model_create and for one grow-only scratch buffer per model, used by
 *    nqs_sample (local energies evaluated after the sweep, and the chains' hidden angles
 *    of float models with more than 256 hidden units), nqs_local_energy and
 *    nqs_log_psi_grad (about n * n_hidden complex values in the compute precision, or
 *    n_chains * n_hidden complex doubles). Growing it allocates and synchronises the
 *    device; calls with one handle must therefore be issued on one stream.
 *  - Calls are asynchronous and ordered on `stream` (a hipStream_t; NULL = the null
 *    stream), except where a call states it synchronises.
 *  - Argument errors are detected on the host before any launch and returned as
 *    NQS_EINVAL (nothing is launched). HIP launch/runtime errors return NQS_EDEVICE.
 *  - A handle must not be used from two threads at once.
 *  - Spins are int8, +1 (up) or -1 (down). Configuration arrays are row-major [n, N].
 *  - RBM parameters are packed p = [a (N) | b (M) | W (M x N, row j, column i)], with
 *    P = N + M + N*M entries (symmetric RBM: see nqs_model_desc), in the model's master
 *    precision: double for NQS_F64, float for NQS_F32 and NQS_BF16; complex models
 *    interleave (re, im) pairs.
 *  - Results that are per-configuration scalars (log psi, local energies, Jacobian
 *    products) and the SR vectors are always double (complex: interleaved double
 *    pairs), whatever the compute precision.
 */
#ifndef NQS_H
#define NQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NQS_OK = 0,
  NQS_ENOTCONV = 1,     /* warning: CG stopped at cg_maxiter before reaching cg_tol */
  NQS_EINVAL = -1,      /* bad argument: null pointer, size out of range, bad enum */
  NQS_ENOMEM = -2,      /* device allocation failed, or workspace too small */
  NQS_EDEVICE = -3,     /* HIP runtime or launch error */
  NQS_ENONFINITE = -4,  /* a NaN/Inf was produced (energy, force or CG scalar) */
  NQS_EUNSUPPORTED = -5 /* valid but not supported combination */
} nqs_status;

/* Precision forms (Sec. 2.2.2 RBM, Sec. 2.2.5 SR; the paper fixes none):
 *  NQS_F64  - every kernel in double.
 *  NQS_F32  - ratio products, local energies, theta/tanh and the Jacobian contractions
 *             in float (matrix cores with float accumulation); hidden angles cached in
 *             double in the sampler; log psi, statistics and the CG solve in double.
 *  NQS_BF16 - the quantised model: every weight W_ji is rounded to the nearest bfloat16
 *             (a, b are not), and the Jacobian contractions of nqs_log_psi_grad and the
 *             SR entry points read tanh(theta) rounded to bfloat16; arithmetic as
 *             NQS_F32. Sampling is exact for the quantised model, so its energies stay
 *             variational. */
typedef enum { NQS_F64 = 0, NQS_F32 = 1, NQS_BF16 = 2 } nqs_prec;
typedef enum { NQS_TFIM = 0, NQS_HEISENBERG = 1 } nqs_hamiltonian;
typedef enum { NQS_MOVE_FLIP = 0, NQS_MOVE_EXCHANGE = 1 } nqs_move;
typedef enum { NQS_ACT_LNCOSH = 0, NQS_ACT_TANH = 1 } nqs_activation;

/*
 * Model description (host memory; everything is copied by nqs_model_create).
 * Sec. 2.2.1: a graph of sites and bonds whose integer color selects the bond type;
 * color 0 = nearest-neighbour bonds (coupling J[0]), color 1 = next-nearest (J[1]).
 *  - NQS_TFIM:       H = -sum_c J[c] sum_{(i,j) in c} sz_i sz_j - h sum_i sx_i
 *  - NQS_HEISENBERG: H = sum_c J[c] sum_{(i,j) in c} (sx sx + sy sy + sz sz)_{ij}
 *    Pauli matrices throughout. With marshall != 0 the Hamiltonian is rotated by
 *    prod_{sublattice[i] = 1} sz_i: the exchange element of bonds joining the two
 *    sublattices changes sign (sublattice must then be given).
 *  - move: NQS_MOVE_FLIP proposes single-spin flips at uniform sites; NQS_MOVE_EXCHANGE
 *    swaps the spins of a uniform color-0 bond (conserves total magnetisation; chains
 *    are initialised at zero magnetisation, so N must be even).
 *  - n_hidden = M hidden units (alpha = M / N); is_complex selects complex parameters.
 *  - n_symm > 0 selects the symmetric RBM (RbmSpinSymm, Sec. 2.2.2): a group of G =
 *    n_symm site permutations, symm [G][n_sites] (host; g maps site i to symm[g][i], and
 *    (T_g sigma)_i = sigma_symm[g][i]), and alpha = M / G filters; hidden unit (f, g)
 *    has theta_fg = b_f + sum_i W_fi sigma_symm[g][i], so psi(T_g sigma) = psi(sigma) when
 *    the permutations form a group. Parameters are then packed p = [a (1) | b (alpha) |
 *    W (alpha x N, row f, column i)], P = 1 + alpha + alpha N (nqs_n_params). Every entry
 *    point of a single model accepts such a model; the batch entry points do not.
 *  - n_layers > 0 selects the feed-forward network (FFNN, Sec. 2.2.2) instead of an RBM:
 *    L = n_layers dense layers, each followed by its activation (layer_sizes[l] outputs,
 *    activations[l] an nqs_activation):
 *      z_0 = sigma, y_l = W_l z_(l-1) + b_l, z_l = f_l(y_l), log psi = sum_k z_L,k,
 *    so that one ln cosh layer is the RBM without visible bias. n_hidden is ignored.
 *    Parameters are packed layer by layer as [b_l (n_l) | W_l (n_l x n_(l-1), row j,
 *    column k)] with n_0 = n_sites. FFNN models run nqs_log_psi, nqs_local_energy,
 *    nqs_sample, nqs_log_psi_grad, nqs_sr_step(_async) and nqs_overlap_step in FP64 or
 *    FP32 (not BF16); the other entry points return NQS_EUNSUPPORTED.
 * Limits: 2 <= n_sites <= 1024, 1 <= n_hidden <= 2048, bonds within [0, n_sites),
 * i != j, n_bonds[0] >= 1 for exchange moves; n_symm divides n_hidden and every row of
 * symm is a permutation of 0 .. n_sites - 1; 1 <= n_layers <= 4 with widths 1 .. 512
 * (not together with n_symm).
 */
typedef struct {
  int32_t n_sites;
  int32_t n_hidden;
  int32_t is_complex;
  int32_t prec;                 /* nqs_prec */
  int32_t n_bonds[2];
  const int32_t *bonds[2];      /* host, [n_bonds[c]][2] site pairs; NULL when n_bonds[c] == 0 */
  int32_t ham;                  /* nqs_hamiltonian */
  double J[2];
  double h;
  int32_t marshall;
  const int8_t *sublattice;     /* host [n_sites], 0/1; required when marshall != 0 */
  int32_t move;                 /* nqs_move */
  int32_t n_symm;               /* 0: RBM; G > 0: symmetric RBM over G site permutations */
  const int32_t *symm;          /* host [n_symm][n_sites]; NULL when n_symm == 0 */
  int32_t n_layers;             /* 0: RBM; 1..4: FFNN with the layers below */
  const int32_t *layer_sizes;   /* host [n_layers]; NULL when n_layers == 0 */
  const int32_t *activations;   /* host [n_layers], nqs_activation */
} nqs_model_desc;

typedef struct nqs_model nqs_model;

/* Information of one SR step (Sec. 2.2.5: the energy is reported with its statistical
 * error and its variance, Fig. 2). nqs_sr_step fills a host struct before it returns;
 * nqs_sr_step_async writes the same struct to device memory, in stream order. */
typedef struct {
  int32_t cg_iters;        /* matrix-vector products performed */
  int32_t converged;       /* 1 if ||r|| <= cg_tol * ||F|| */
  double cg_resid;         /* final recursive residual ||r|| / ||F|| */
  double energy_re, energy_im;  /* mean local energy */
  double variance;         /* mean |E_loc - E|^2 */
  double force_norm;       /* ||F||_2 */
  double energy_err;       /* error bar of energy_re: with C chains and the samples laid out
                              [sweeps, chains], m_c = mean of Re E_loc over chain c and
                              energy_err = sqrt(sum_c (m_c - mean m)^2 / (C - 1)) / sqrt(C);
                              n_chains = 0 treats every sample as its own chain */
  int32_t status;          /* NQS_OK, NQS_ENOTCONV or NQS_ENONFINITE: the step's outcome */
  int32_t reserved;
} nqs_sr_info;

/* Lattice helper (Sec. 2.2.1, Hypercube graph): periodic L^ndim hypercube, ndim 1 or 2.
 * Site s = x0 + L*x1. Color-0 bonds are listed site by site, dimension by dimension, as
 * (s, s + e_d); color-1 (ndim = 2 and with_diagonals) as (s, s+ex+ey), (s, s+ex-ey).
 * sublattice[s] = (x0 + x1) mod 2. Outputs are host arrays sized by the caller:
 * bonds0 [ndim*L^ndim][2], bonds1 [2*L^2][2] (may be NULL without diagonals),
 * sublattice [L^ndim]; n_bonds[2] receives the counts. Requires 3 <= L <= 1024. */
nqs_status nqs_hypercube(int32_t L, int32_t ndim, int32_t with_diagonals, int32_t *bonds0,
                         int32_t *bonds1, int8_t *sublattice, int32_t *n_bonds);

/* The L^ndim translations of the periodic hypercube of nqs_hypercube as site
 * permutations (the symmetry group of a symmetric RBM on it): perm (host) [L^ndim][L^ndim]
 * receives perm[g][s] = site s moved by the lattice vector of site g (g = 0 is the
 * identity). Requires 3 <= L and L^ndim <= 1024. */
nqs_status nqs_hypercube_translations(int32_t L, int32_t ndim, int32_t *perm);

/* Create a model handle: validates the description and uploads the bond tables. */
nqs_status nqs_model_create(const nqs_model_desc *desc, nqs_model **out);
void nqs_model_destroy(nqs_model *model);
int64_t nqs_n_params(const nqs_model *model);

/* Chain initialisation (Sec. 2.2.5 sampler set-up). chain_sigma (device) [n_chains, N]
 * receives independent +/-1 spins (flip moves) or a uniformly random permutation of
 * N/2 up and N/2 down spins (exchange moves), drawn from Philox4x32-10 with key = seed
 * and counter (chain_offset + c, 0, site, 1). */
nqs_status nqs_chain_init(nqs_model *model, int8_t *chain_sigma, int32_t n_chains,
                          uint64_t seed, int32_t chain_offset, void *stream);

/* Metropolis sampling of pi(sigma) = |psi|^2 / sum |psi|^2 (Sec. 2.2.5, Eq. 4).
 * Every chain runs n_discard + n_sweeps sweeps of N proposals. Proposal `step` of sweep
 * `sw` of chain c draws Philox4x32-10 with key = seed and counter
 * (chain_offset + c, counter + sw, step, 0): word 0 picks the site (flip) or color-0
 * bond (exchange) as floor(w0 * n / 2^32); words 1, 2 give u = (w1 * 2^21 + w2 >> 11)
 * * 2^-53. Accept iff |psi'/psi|^2 >= 1 or u < |psi'/psi|^2. NQS_F64 takes this
 * decision in double: the wave product of the ratio terms as mantissa x 2^exponent,
 * scaled by |exp(visible-bias change)|^2 and compared with u. NQS_F32 and NQS_BF16 take
 * it in the float log domain: each lane forms log2 of the product of |ratio term|^2 of
 * up to four of its hidden units (hardware log2), the wavefront sums these in float, and
 * the proposal is accepted iff the sum exceeds log2(u) - log2|exp(visible-bias
 * change)|^2 (also float). This agrees with the exact rule except within a relative
 * margin of about 1e-5 around |psi'/psi|^2 = u (the parity tests allow a chain to leave
 * the FP64 oracle's chain only after a proposal with |u - |psi'/psi|^2| < 1e-4). An
 * exchange of equal spins is an identity move (not counted). After each of the last
 * n_sweeps sweeps the configuration is written to samples[sweep][c][:].
 *  params      (device) packed RBM parameters (master precision; see top)
 *  chain_sigma (device) [n_chains, N] in: current chains, out: chains after the call
 *  samples     (device) [n_sweeps, n_chains, N]
 *  n_accepted  (device) int64 [n_chains] accepted proposals in this call (may be NULL)
 *  eloc        (device) double/complex double [n_sweeps * n_chains] or NULL: if given,
 *              the local energy of every recorded sample (same values as
 *              nqs_local_energy on `samples`, up to rounding). With at least 16 chains per
 *              compute unit and at most 256 hidden units it is evaluated inside the sweep
 *              from the chain's cached hidden-unit angles; otherwise by a separate pass
 *              over the samples.
 * Limits: n_chains >= 1, n_sweeps >= 1, n_discard >= 0, chain_offset >= 0. */
nqs_status nqs_sample(nqs_model *model, const void *params, int8_t *chain_sigma,
                      int32_t n_chains, int32_t n_sweeps, int32_t n_discard, uint64_t seed,
                      uint64_t counter, int32_t chain_offset, int8_t *samples,
                      int64_t *n_accepted, void *eloc, void *stream);

/* Metropolis sampling with parallel tempering (Sec. 2.2.5: the samplers' tempering
 * option). Each of the n_chains chains carries R = n_replicas replicas (2 <= R <= 16);
 * replica w of chain c is row c R + w of chain_sigma (device [n_chains, R, N], in/out) and
 * holds the temperature index temp_index[c R + w] (device int32, in/out; the indices of a
 * chain are a permutation of 0 .. R-1, e.g. w at the first call), i.e. it samples
 * |psi|^(2 beta) with beta_r = 1 - r / R. A sweep runs N proposals in every replica, drawn
 * as in nqs_sample with chain index (chain_offset + c) R + w and accepted iff
 * |psi'/psi|^(2 beta) >= 1 or u < |psi'/psi|^(2 beta). After each sweep the temperatures
 * k and k + 1 are exchanged, for k = 0 .. R-2 in order, iff E >= 0 or u < exp(E) with
 * E = (beta_k - beta_k+1)(L_b - L_a), L = 2 Re log psi (in double, from the replicas'
 * exact angles) of the replicas a, b holding k, k + 1, and u from Philox4x32-10 counter
 * (chain_offset + c, counter + sweep, k, 2). After each of the last n_sweeps sweeps the
 * configuration of the replica holding beta = 1 is written to samples[sweep][c][:]
 * (device [n_sweeps, n_chains, N]). n_accepted (device int64 [n_chains R], may be NULL):
 * accepted proposals per replica; n_swaps (device int64 [n_chains], may be NULL): accepted
 * exchanges; eloc (device [n_sweeps n_chains], may be NULL): local energies of the recorded
 * samples. One block per chain, one wavefront per replica (hence R <= 4); float models with
 * more than 256 hidden units are not tempered (NQS_EUNSUPPORTED). */
nqs_status nqs_sample_pt(nqs_model *model, const void *params, int8_t *chain_sigma,
                         int32_t *temp_index, int32_t n_chains, int32_t n_replicas,
                         int32_t n_sweeps, int32_t n_discard, uint64_t seed, uint64_t counter,
                         int32_t chain_offset, int8_t *samples, int64_t *n_accepted,
                         int64_t *n_swaps, void *eloc, void *stream);

/* ---- Supervised learning (Sec. 2.2.3): the negative log overlap of Eq. 1 with a target
 * state t, minimised by the update of Eq. 2 from configurations drawn from |t|^2. ----
 *
 * Targets are given on a training set of n_states configurations (states, device int8
 * [n_states, N], +1/-1) with log t (device, the model's value type: complex double [n_states]
 * re/im interleaved for complex models, double for real models, i.e. positive targets).
 *
 * nqs_target_cdf: cdf[k] = sum_{i <= k} |t_i|^2 / max_i |t_i|^2 (device double [n_states],
 * summed in a fixed order). */
nqs_status nqs_target_cdf(nqs_model *model, const void *log_target, int64_t n_states,
                          double *cdf, void *stream);

/* nqs_target_draw: n direct draws from |t|^2: draw s takes the Philox4x32-10 uniform u of
 * counter (s, counter, 0, 3) under key seed and picks the first k with cdf[k] > u cdf_last;
 * it writes the configuration to sigma[s] (device int8 [n, N]), log t_k to
 * log_target_out[s] (device, value type [n]) and k to index[s] (device int64 [n], may be
 * NULL). */
nqs_status nqs_target_draw(nqs_model *model, const double *cdf, int64_t n_states,
                           const int8_t *states, const void *log_target, int64_t n,
                           uint64_t seed, uint64_t counter, int8_t *sigma, void *log_target_out,
                           int64_t *index, void *stream);

/* Result of one supervised step (host memory). */
typedef struct {
  double loss;       /* Monte Carlo estimate of Eq. 1: -log(|sum conj R|^2 / (n sum |R|^2)),
                        R_s = psi(sigma_s) / t(sigma_s) */
  double overlap;    /* exp(-loss) */
  double grad_norm;  /* ||g||_2 of the gradient below */
  int32_t status;    /* NQS_OK, or NQS_ENONFINITE (parameters left unchanged) */
  int32_t reserved;
} nqs_overlap_info;

/* nqs_overlap_step: one step of Eq. 2 from n >= 1 samples sigma (device int8 [n, N]) drawn
 * from |t|^2, with their log t (device, value type [n]): p <- p - lr g with
 * g = dL/dconj(p) = O^dagger u, u_s = |R_s|^2 / sum |R|^2 - conj(R_s) / sum conj(R)
 * (for real parameters the real part, half of dL/dp: the convention of the SR force).
 * params: device, the model's parameter type, updated in place unless the loss or the
 * gradient is not finite. Uses the model's scratch (allocated on first use); synchronises
 * the stream to fill info (host, may be NULL). */
nqs_status nqs_overlap_step(nqs_model *model, void *params, const int8_t *sigma,
                            const void *log_target, int64_t n, double lr,
                            nqs_overlap_info *info, void *stream);

/* log psi(sigma) = sum_i a_i sigma_i + sum_j ln cosh(theta_j), theta = W sigma + b
 * (Sec. 2.2.2: RBM as a one-layer ln cosh network plus visible bias; the constant
 * M ln 2 of prod_j 2 cosh is dropped). sigma (device) [n, N]; logpsi (device) [n]
 * double or complex double (imaginary part defined modulo 2 pi). n >= 0. */
nqs_status nqs_log_psi(nqs_model *model, const void *params, const int8_t *sigma, int64_t n,
                       void *logpsi, void *stream);

/* Local energy, Eq. 5: E_loc(sigma) = sum_sigma' <sigma|H|sigma'> psi(sigma')/psi(sigma)
 * over the configurations connected to sigma. sigma (device) [n, N]; eloc (device) [n]
 * double (real model) or complex double. n >= 0. */
nqs_status nqs_local_energy(nqs_model *model, const void *params, const int8_t *sigma,
                            int64_t n, void *eloc, void *stream);

/* Jacobian products of O_sk = d log psi(sigma_s) / d p_k (Sec. 2.2.5, analytic RBM
 * derivatives: O_a = sigma, O_b = tanh theta, O_W = tanh(theta) sigma):
 *   vjp[k] = sum_s conj(O_sk) u[s]     (if u and vjp are both non-NULL)
 *   jvp[s] = sum_k O_sk v[k]           (if v and jvp are both non-NULL)
 * theta is recomputed from sigma (nothing is stored between calls). u, jvp: (device)
 * [n]; v, vjp: (device) [P]; all double / complex double. The contractions run in the
 * model precision (FP64, FP32 or BF16 inputs with FP32 accumulation). */
nqs_status nqs_log_psi_grad(nqs_model *model, const void *params, const int8_t *sigma,
                            int64_t n, const void *u, void *vjp, const void *v, void *jvp,
                            void *stream);

/* nqs_log_psi_grad for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation): the same products,
 * arguments and results (bit for bit), with the call's scratch (tanh(theta) rows,
 * direction tables, partial tiles) in one fixed 64 MiB array per device that the library
 * holds for the life of the process, instead of the model's grow-only buffer. The call
 * allocates and frees nothing and never synchronises. Returns NQS_ENOMEM, before any
 * launch, when the scratch these n samples need exceeds 64 MiB (about 19 MB of partial
 * tiles plus 680 bytes per sample for a complex FP32 model with N = 40, M = 80: some
 * 70,000 samples); the first call on a device looks up the array's address there. Every call on one device shares that
 * device's array, which keeps the last call's contents: calls that overlap on one device
 * (other streams or threads) race and must be ordered by the caller. */
nqs_status nqs_log_psi_grad_noalloc(nqs_model *model, const void *params, const int8_t *sigma,
                                    int64_t n, const void *u, void *vjp, const void *v,
                                    void *jvp, void *stream);

/* Device workspace (bytes) needed by nqs_sr_step for n samples. */
size_t nqs_sr_workspace_bytes(nqs_model *model, int64_t n);

/* One stochastic-reconfiguration update (Sec. 2.2.5; the parameter step of Eq. 2):
 *   E = <E_loc>, F_k = <conj(O_k)(E_loc - E)>, S_kk' = <conj(O_k) O_k'> - <conj O_k><O_k'>
 *   solve (S + diag_shift I) x = F by conjugate gradients in double (x0 = 0, stop when
 *   ||r|| <= cg_tol ||F|| or after cg_maxiter products), S applied implicitly as
 *   S v = O^dagger (O v - mean(O v)) / n, then params <- params - lr x.
 * Real models use real arithmetic throughout. params (device) in/out; sigma (device)
 * [n, N]; eloc (device) [n] double/complex double; n_chains: the samples are laid out
 * [n / n_chains sweeps, n_chains chains] for the energy error bar (n_chains divides n;
 * 0 = every sample its own chain); workspace (device) of at least
 * nqs_sr_workspace_bytes(model, n) bytes; info (host) may be NULL.
 * Synchronises `stream` (the CG loop checks convergence on the host every few
 * iterations, while the next chunk of iterations already runs). Returns NQS_ENOTCONV if
 * cg_maxiter was reached, NQS_ENONFINITE if the energy, the force or a CG scalar is not
 * finite (params are then left unchanged).
 * Limits: n >= 2, 0 <= n_chains <= n, cg_maxiter >= 1, cg_tol >= 0, diag_shift >= 0. */
nqs_status nqs_sr_step(nqs_model *model, void *params, const int8_t *sigma, const void *eloc,
                       int64_t n, int32_t n_chains, double lr, double diag_shift,
                       double cg_tol, int32_t cg_maxiter, void *workspace, size_t ws_bytes,
                       nqs_sr_info *info, void *stream);

/* The same SR update, stream-ordered (Sec. 2.2.5, Eq. 2): nothing is read back on the
 * host, so the call returns after queueing its kernels and may be captured into a
 * hipGraph. The solve runs exactly cg_maxiter iteration slots; convergence (or a
 * non-finite scalar) is decided on the device, and the slots after it return at once,
 * so cg_maxiter is the caller's bound on the work queued (a solve that needs more
 * iterations ends with NQS_ENOTCONV in info->status). The parameters are updated on the
 * device only when the energy, the force and every CG scalar are finite. info (device)
 * receives the step's nqs_sr_info, status included. Results equal those of nqs_sr_step
 * with the same arguments bit for bit. The call allocates nothing, copies nothing and
 * never synchronises.
 * Returns NQS_EINVAL / NQS_ENOMEM / NQS_EDEVICE for argument and launch errors only. */
nqs_status nqs_sr_step_async(nqs_model *model, void *params, const int8_t *sigma,
                             const void *eloc, int64_t n, int32_t n_chains, double lr,
                             double diag_shift, double cg_tol, int32_t cg_maxiter,
                             void *workspace, size_t ws_bytes, nqs_sr_info *info,
                             void *stream);

/* The S v product of stochastic reconfiguration on its own (Sec. 2.2.5; the implicit form
 * S v = O^dagger (O v - mean(O v)) / n of the same S as nqs_sr_step), for custom solvers
 * and for measurement. nqs_sr_prepare computes tanh(theta) of every sample and
 * O^dagger 1 into `workspace` (nqs_sr_workspace_bytes(model, n) bytes) from params and
 * sigma [n, N]; then each nqs_sr_matvec writes out = (S + diag_shift I) v for v, out
 * (device) [P] double / complex double, reusing the prepared workspace (the sigma passed
 * must be the same). The workspace holds the preparation until it is reused by another
 * call. Limits: n >= 2, diag_shift >= 0. */
nqs_status nqs_sr_prepare(nqs_model *model, const void *params, const int8_t *sigma, int64_t n,
                          void *workspace, size_t ws_bytes, void *stream);
nqs_status nqs_sr_matvec(nqs_model *model, const int8_t *sigma, int64_t n, void *workspace,
                         size_t ws_bytes, const void *v, double diag_shift, void *out,
                         void *stream);

/* Tile-shape autotuner for the S v product of stochastic reconfiguration (the contraction
 * that dominates an SR step, Sec. 2.2.5). Times every kernel shape that applies to this
 * model at this sample count (n samples sigma [n, N] on the device, parameters params)
 * with one prepared workspace (nqs_sr_workspace_bytes(model, n) bytes), ten products
 * each, and keeps the fastest in the model for all later calls. Workspace sizes do not
 * depend on the shape chosen. Synchronizes the stream. report (host, may be NULL)
 * receives the candidates and their mean times. The product's result differs between
 * shapes only by floating-point summation order. */
#define NQS_TUNE_MAX 4
typedef struct {
  int32_t n_candidates;          /* shapes timed (1 when the model has no choice) */
  int32_t chosen;                /* index of the shape kept */
  int32_t pairs[NQS_TUNE_MAX];   /* wavefront pairs per block of each candidate */
  double us[NQS_TUNE_MAX];       /* mean microseconds of one S v product */
} nqs_tune_report;
nqs_status nqs_autotune(nqs_model *model, const void *params, const int8_t *sigma, int64_t n,
                        void *workspace, size_t ws_bytes, nqs_tune_report *report,
                        void *stream);
/* Re-applies a shape the autotuner chose earlier (report.pairs[report.chosen]) without
 * timing again; 2 or 4, otherwise NQS_EINVAL. Models where the shape does not apply
 * ignore it. */
nqs_status nqs_set_sv_shape(nqs_model *model, int32_t pairs);

/* nqs_sr_step launches its CG iterations in chunks of 8 and, by default, replays full
 * chunks from a graph captured on the first chunk (re-captured when the workspace,
 * samples, n, shift, tolerance, iteration limit or S v shape change); the results are
 * those of the plain launches. enable = 0 launches every kernel directly (for callers
 * that capture the whole step into a graph of their own). */
nqs_status nqs_set_cg_graphs(nqs_model *model, int32_t enable);

/* Timing of one kind of kernel launch, for measurement (no effect on results): while
 * what != NQS_TIME_NONE the model records pairs of HIP events on the launch stream right
 * before and right after the kernels of that kind in each call, and nqs_kernel_ms returns
 * the sum of the times between the pairs of the last such call (it waits for them).
 *  NQS_TIME_SWEEP - the Metropolis sweep kernel of nqs_sample (not the table refresh, the
 *                   chain-angle set-up or local energies evaluated after the sweep)
 *  NQS_TIME_SV    - the kernels of one nqs_sr_matvec product (direction tables, the
 *                   contractions, the reduced product), without the gaps between them;
 *                   for a feed-forward network the O^dagger u and O v kernels of one
 *                   nqs_log_psi_grad call (not its forward-backward pass)
 *  NQS_TIME_ELOC  - the local-energy kernel of nqs_local_energy (not tanh(theta)) */
typedef enum { NQS_TIME_NONE = 0, NQS_TIME_SWEEP = 1, NQS_TIME_SV = 2, NQS_TIME_ELOC = 3 } nqs_time_what;
nqs_status nqs_time_kernel(nqs_model *model, int32_t what);
nqs_status nqs_kernel_ms(nqs_model *model, float *ms);
/* The individual pairs of the last timed call, in launch order: ms[k] (host, k < cap) for
 * k < *count (host; at most 8 pairs are recorded per call). For NQS_TIME_SV the pairs of
 * one nqs_sr_matvec product are, in order: the direction tables, the O v kernels, the
 * O^dagger y kernel (the fused S v kernel, for shapes that fuse both), the reduction into
 * (S + lambda I) v. */
nqs_status nqs_kernel_times(nqs_model *model, float *ms, int32_t cap, int32_t *count);

/* ---- Batches of independent models (uneven sizes) --------------------------------
 * A batch holds K models created from K descriptions (all with the same is_complex and
 * prec; sizes, Hamiltonians, couplings and moves may differ). Buffers of the models are
 * concatenated in model order, each in the layout of the single-model call:
 *   params      model k at element offset sum_{i<k} P_i (P_i = nqs_batch_n_params(i))
 *   chain_sigma model k at byte offset sum_{i<k} C_i N_i          ([C_k, N_k])
 *   samples     model k at byte offset n_sweeps sum_{i<k} C_i N_i  ([n_sweeps, C_k, N_k])
 *   eloc        model k at element offset n_sweeps sum_{i<k} C_i  ([n_sweeps * C_k])
 *   n_accepted  model k at offset sum_{i<k} C_i
 * n_chains is a host array [K]. Model k draws its random numbers with seed ^ k: its
 * chains and samples equal those of nqs_chain_init / nqs_sample on its own model with
 * that seed and chain_offset 0. Sampling (Sec. 2.2.5) runs every chain of every model in
 * one persistent launch, after one launch that refreshes every model's tables; local
 * energies (Eq. 5) are evaluated inside the sweep when eloc is not NULL. counter_dev
 * (device, one uint64, may be NULL): when given, the sweep base of the counter is read
 * from it on the device (the counter argument is then ignored) and advanced by
 * n_discard + n_sweeps after the sweeps, in stream order, so that replays of a captured
 * call continue the random stream as consecutive calls would. The block-to-model tables
 * are uploaded (synchronously) only when buffers or sizes change (not the counter), so a
 * repeated call with the same buffers issues no host-to-device copy and can be captured
 * into a hipGraph after one uncaptured call. */
typedef struct nqs_batch nqs_batch;
nqs_status nqs_batch_create(const nqs_model_desc *descs, int32_t n_models, nqs_batch **out);
void nqs_batch_destroy(nqs_batch *batch);
int64_t nqs_batch_n_params(const nqs_batch *batch, int32_t k);
nqs_status nqs_batch_chain_init(nqs_batch *batch, int8_t *chain_sigma, const int32_t *n_chains,
                                uint64_t seed, void *stream);
nqs_status nqs_batch_sample(nqs_batch *batch, const void *params, int8_t *chain_sigma,
                            const int32_t *n_chains, int32_t n_sweeps, int32_t n_discard,
                            uint64_t seed, uint64_t counter, uint64_t *counter_dev,
                            int8_t *samples, int64_t *n_accepted, void *eloc, void *stream);
/* One SR step (Sec. 2.2.5, Eq. 2) of every model of the batch, as nqs_sr_step on each:
 * samples and eloc concatenated in model order (model k: n_samples[k] rows of N_k spins,
 * n_samples[k] local energies, laid out [sweeps, n_chains[k]] for the error bar;
 * n_chains (host [K]) may be NULL: every sample its own chain), params updated in place,
 * info (host) an array [K]. The solves advance together: every kernel of a CG iteration
 * is one launch for all models, and models that have converged stop updating. Returns
 * NQS_ENONFINITE if any model's solve is non-finite (its parameters are left unchanged),
 * else NQS_ENOTCONV if any model reached cg_maxiter, else NQS_OK. Synchronizes the
 * stream. Workspace: nqs_batch_sr_workspace_bytes(batch, n_samples) bytes (0 if some
 * n_samples[k] < 2). */
size_t nqs_batch_sr_workspace_bytes(nqs_batch *batch, const int64_t *n_samples);
nqs_status nqs_batch_sr_step(nqs_batch *batch, void *params, const int8_t *samples,
                             const void *eloc, const int64_t *n_samples,
                             const int32_t *n_chains, double lr, double diag_shift,
                             double cg_tol, int32_t cg_maxiter, void *workspace,
                             size_t ws_bytes, nqs_sr_info *info, void *stream);
/* The batched SR step, stream-ordered (Sec. 2.2.5, Eq. 2): as nqs_sr_step_async for every
 * model of the batch (cg_maxiter iteration slots, convergence decided per model on the
 * device, parameters updated only where finite), info (device) an array [K] of
 * nqs_sr_info. Results equal those of nqs_batch_sr_step bit for bit. The job tables that
 * map blocks to models are uploaded (synchronously) only when buffers or sizes change, so
 * after one call with the same arguments the call queues kernels only and can be
 * captured into a hipGraph, together with nqs_batch_sample. A captured graph reads the
 * job tables of its batch handle: calls on that handle with other buffers or sizes
 * rewrite them, so give each captured pipeline a handle of its own. */
nqs_status nqs_batch_sr_step_async(nqs_batch *batch, void *params, const int8_t *samples,
                                   const void *eloc, const int64_t *n_samples,
                                   const int32_t *n_chains, double lr, double diag_shift,
                                   double cg_tol, int32_t cg_maxiter, void *workspace,
                                   size_t ws_bytes, nqs_sr_info *info, void *stream);

const char *nqs_status_string(nqs_status s);

#ifdef __cplusplus
}
#endif
#endif /* NQS_H */
