/*
 * libthcsox -- second-order exchange (SOX) self-energy with tensor-hypercontracted
 * Coulomb integrals, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Pokhilko, Yeh, Morales, Zgid, "Tensor hypercontraction for fully
 * self-consistent imaginary-time GF2 and GWSOX methods", Sec. "THC-scGF2:
 * algorithm and implementation details" (the SOX expression and the THC
 * contraction sequence that starts with Eq. U_contraction), with the
 * integrals in the factorised form of Eq. THC_ERI:
 *     (ij|kl) = sum_PQ X_iP X_jP V_PQ X_kQ X_lQ        (real X, symmetric V)
 * and the energy of Eq. E2b (Sec. "Definitions").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array is row-major and FP64 at the boundary.  "dev" pointers must be
 *    device memory of the current HIP device, "host" pointers host memory; a
 *    wrong kind is rejected with THCSOX_ENOTDEV before any work is queued.
 *  - n = number of orbitals, naux = number of THC points, ntau = number of
 *    imaginary-time points.  G[k][p][q] = G_pq(tau_k).
 *  - The tau grid must be ascending inside (0, beta) and mirror symmetric,
 *    |tau_k + tau_{ntau-1-k} - beta| <= 1e-12 beta, so that the value the SOX
 *    expression needs at -tau_k is read from index ntau-1-k (it is taken as
 *    G(beta - tau_k), keeping the expression's leading minus sign).
 *  - Work is queued on the plan's stream (the stream given to thcsox_plan, or the
 *    null stream) and is asynchronous unless stated otherwise.
 *  - Return value: 0 on success, a negative THCSOX_E* code on failure; the
 *    message of the last failure on the calling thread is in thcsox_last_error().
 *    No C++ exception crosses this interface.
 *  - One plan must not be used from two threads at once; distinct plans are
 *    independent.
 */
#ifndef THCSOX_H
#define THCSOX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic of the contraction stages (the boundary is always FP64).  The
 * projections, back-projection and energy always run in FP64.
 *   FP64   : FP64 matrix cores.
 *   FP32   : FP32 matrix cores, FP32 accumulation.
 *   BF16X3 : every operand split into three bfloat16 terms, six products per
 *            product kept, FP32 accumulation.
 *   FP16X2 : every operand scaled by a power of two and split into two
 *            half-precision terms, three products per product, FP32 accumulation
 *            (the intermediate A, formed on the device, takes its power of two
 *            from a Cauchy-Schwarz bound computed before it is formed).
 * In every mode G is scaled per tau point by a power of two.  The sum over the
 * orbital index v that forms D_PR is accumulated in FP64 by the FP64 mode; the
 * other modes sum at most 8 consecutive v in FP32, then add those partial sums
 * in FP64 (FP32 partial tiles when a v range holds at most 8 v, summed over
 * the ranges in FP64). */
enum {
  THCSOX_FP64 = 0,
  THCSOX_FP32 = 1,
  THCSOX_BF16X3 = 2,
  THCSOX_FP16X2 = 3
};

enum {
  THCSOX_OK = 0,
  THCSOX_EINVAL = -1,     /* bad sizes, grid, precision or index range */
  THCSOX_ENOMEM = -2,     /* device allocation failed or workspace_limit too small */
  THCSOX_EDEVICE = -3,    /* a HIP call failed; message carries hipGetErrorString */
  THCSOX_ENONFINITE = -4, /* NaN/Inf found in an input (only where checks are on) */
  THCSOX_ENOTDEV = -5     /* a host pointer where device memory is required (or v.v.) */
};

typedef struct thcsox_plan_s* thcsox_plan_t;

/* Build a plan for one system and precompute
 *     U_Pqs = sum_Q V_PQ X_qQ X_sQ                   (Eq. U_contraction)
 * once, in FP64 (stored in the plan's contraction precision).
 *   out            : receives the plan handle (host pointer).
 *   n, naux, ntau  : > 0.
 *   beta           : inverse temperature, > 0.
 *   tau_host[ntau] : ascending, mirror-symmetric grid in (0, beta).
 *   wq_host[ntau]  : quadrature weights on [0, beta] used by thcsox_energy.
 *   X_dev[n][naux], V_dev[naux][naux] : THC factors (V symmetric).  Copied:
 *                    the caller may free them when this call returns.
 *   precision      : one of THCSOX_FP64 .. THCSOX_FP16X2.  The fused kernels
 *                    address one tile's rows of U with 32-bit buffer offsets,
 *                    which bounds n: n <= 2047 (FP64, FP32), 2880 (BF16X3,
 *                    one resource per plane), 2047 (FP16X2, whose rows hold
 *                    both planes); larger n is THCSOX_EINVAL.
 *   workspace_limit: upper bound in bytes on everything the plan allocates,
 *                    the temporaries of building U (freed before this call
 *                    returns) included (0 = no bound).  The number of tau
 *                    points processed per batch shrinks to fit; THCSOX_ENOMEM
 *                    if one does not fit.
 *   hip_stream     : hipStream_t to queue work on (NULL = null stream).
 * Synchronises the stream before returning.  The plan owns all its memory. */
int thcsox_plan(thcsox_plan_t* out, int n, int naux, int ntau, double beta,
                const double* tau_host, const double* wq_host,
                const double* X_dev, const double* V_dev, int precision,
                size_t workspace_limit, void* hip_stream);

/* Sigma^SOX(tau_k) for k in [k_begin, k_end) -- the THC sequence of the paper
 * (Eq. U_contraction and the equations that follow it):
 *     G_Rq  = sum_u X_uR G_uq(tau)        G_wP = sum_p G_wp(tau) X_pP
 *     A_Pqv = sum_s U_Pqs G_sv(-tau)      B_PRv = sum_q A_Pqv G_Rq
 *     C_RvP = sum_w U_Rvw G_wP            D_PR = sum_v C_RvP B_PRv
 *     Sig_RP = -D_PR                      Sigma_tr = sum_PR X_tR Sig_RP X_rP
 *   G_dev[ntau][n][n]          : Green's function on the whole grid (read).
 *   Sigma_dev[ntau][n][n]      : slots k_begin..k_end-1 are written.
 *   Sigma_thc_dev[ntau][naux][naux] : optional (NULL to skip); slots
 *                    k_begin..k_end-1 receive Sig_RP (as computed above; it is
 *                    not unique, X has rank <= n).
 * Symmetric inputs: when G(tau_k) and G(beta - tau_k) are both symmetric to
 * within 1e-12 (FP64 plans) or 1e-10 (the other precisions, whose own rounding
 * is about 1e-8) of the largest element of G on the grid (checked on the
 * device at every call, see thcsox_set_symmetry), D_PR = D_RP holds (U_Pqs = U_Psq by construction),
 * so only tiles of D touching the upper triangle are formed and the rest is
 * mirrored; Sigma changes by at most about that relative asymmetry.
 * 0 <= k_begin < k_end <= ntau.  Sigma must not alias G.  Asynchronous. */
int thcsox_sigma_sox(thcsox_plan_t p, const double* G_dev, double* Sigma_dev,
                     double* Sigma_thc_dev, int k_begin, int k_end);

/* Use of the symmetry of D described at thcsox_sigma_sox:
 *   THCSOX_SYM_AUTO (default): per tau point, where the inputs are symmetric;
 *   THCSOX_SYM_OFF: never (every tile of D is formed).
 * Synchronises the plan's stream.  THCSOX_EINVAL for another mode. */
enum { THCSOX_SYM_AUTO = 0, THCSOX_SYM_OFF = 1 };
int thcsox_set_symmetry(thcsox_plan_t p, int mode);

/* flags_host[ntau]: 1 for each tau point the last thcsox_sigma_sox call would
 * (or did) take the symmetric path for, 0 otherwise (all 0 under
 * THCSOX_SYM_OFF).  Synchronises the plan's stream. */
int thcsox_symmetric_flags(thcsox_plan_t p, int* flags_host);

/* Galitskii-Migdal dynamic energy of Eq. E2b, read as the spin-orbital form
 * with a factor 1/2 and evaluated on the tau grid:
 *     E = -1/2 sum_k w_k Tr[G(beta - tau_k) Sigma(tau_k)],  G(beta-tau_k) = G[ntau-1-k]
 * accumulated in FP64 in a fixed order (bitwise reproducible).
 *   G_dev, Sigma_dev : [ntau][n][n] device arrays.   E_host : host scalar.
 * Synchronises the plan's stream. */
int thcsox_energy(thcsox_plan_t p, const double* G_dev, const double* Sigma_dev,
                  double* E_host);

/* Allocation-free variant of thcsox_energy, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  No plan: the quadrature weights come as a device
 * array.  Computes the same E with the same kernels and summation order as
 * thcsox_energy (bit-identical for the same inputs and weights):
 *   G_dev, Sigma_dev : [ntau][n][n] device arrays (inputs, caller-owned).
 *   w_dev[ntau]      : device array of quadrature weights (input).
 *   E_dev            : one device double (output); written on the stream.
 *   hip_stream       : stream of the current device (NULL: the null stream).
 * The per-tau traces go to a fixed device scratch of at most 4096 doubles
 * that each GPU holds for the life of the process; ntau > 4096 gives
 * THCSOX_EINVAL.  Calls no allocator and does not synchronise (asynchronous;
 * the caller synchronises before reading E_dev).  Every call on one GPU shares
 * that scratch, so calls that overlap in time on one GPU (on different
 * streams, or from different threads) race; calls ordered on one stream are
 * safe.  THCSOX_ENOTDEV for a host pointer, THCSOX_EINVAL for a stream of
 * another device. */
int thcsox_energy_noalloc(const double* G_dev, const double* Sigma_dev, const double* w_dev,
                          int n, int ntau, double* E_dev, void* hip_stream);

/* The same energy on a grid whose quadrature is a basis expansion (the IR
 * sampling grid of thcsox_ir_create): with coefficients g = C G(tau),
 * sigma = C Sigma(tau) (C: coef_host [ntau][ntau], row l maps the tau values to
 * coefficient l) and u_l(beta - tau) = sign_l u_l(tau) for an orthonormal basis,
 *     E = -1/2 int_0^beta Tr[G(beta - tau) Sigma(tau)] dtau
 *       = -1/2 sum_l sign_l sum_pq g_l[p][q] sigma_l[q][p].
 * The plan's tau points must be the basis's sampling points (mirror-symmetric,
 * so that the SOX evaluation finds G(beta - tau_k) at index ntau-1-k).  The
 * first call allocates 2 ntau n^2 doubles (kept by the plan).  FP64, fixed
 * summation order; synchronises the plan's stream. */
int thcsox_energy_basis(thcsox_plan_t p, const double* G_dev, const double* Sigma_dev,
                        const double* coef_host, const double* sign_host, double* E_host);

/* The second-order direct (bubble) self-energy of GF2 on the same THC data
 * (Sec. "Self-energy functionals": full scGF2 = direct + SOX terms; the paper
 * treats this term as in the THC-GW work it cites and prints no formula).
 * Definition, in the spin-orbital convention of the SOX term and with G(-tau)
 * read as G(beta - tau) = G[ntau-1-k]:
 *     Sigma^dir_tr = + sum_{pqsuvw} (tu|vw) (pr|qs) G_up G_wq G_sv(-tau)
 * computed in THC form in FP64 for every plan precision:
 *     Gt = X^T G[k] X, Gbt = X^T G[ntau-1-k] X, Pi_QS = Gt_QS Gbt_SQ,
 *     W = V Pi V, Sigma^dir[k] = X (W o Gt) X^T      (2 naux^3 + O(naux^2 n) per tau)
 * for k in [k_begin, k_end).  G_dev, Sigma_dev: [ntau][n][n] device arrays (Sigma
 * must not alias G).  accumulate = 0 writes Sigma[k]; accumulate = 1 adds to it
 * (e.g. onto the SOX term from thcsox_sigma_sox, giving the full second-order
 * scGF2 self-energy).  The first call allocates 3 x 8 naux^2 bytes per tau point
 * of its batch (about 1 GB at most; counted against workspace_limit).
 * Asynchronous on the plan's stream.  The energy of either term (or of their
 * sum) is thcsox_energy of that Sigma. */
int thcsox_sigma_direct(thcsox_plan_t p, const double* G_dev, double* Sigma_dev, int k_begin,
                        int k_end, int accumulate);

/* The statically screened interaction on the THC grid, for the screened
 * exchange terms below.  The paper names second-order screened exchange (one
 * screened interaction line) and G3W2 (two) as contractions of the SOX type
 * (closing paragraph of Sec. "THC-scGF2: algorithm and implementation details";
 * Sec. "Conclusions and future work") and prints no formula.  Reading used:
 * the polarization is the direct term's bubble and the line is screened in the
 * random-phase series at zero bosonic frequency,
 *     Pi(tau)_QS = Gt_QS Gbt_SQ,   Pi0 = sum_k w_k Pi(tau_k)  (the plan's weights),
 *     W = (1 + V Pi0)^-1 V  (= V - V Pi0 V + V Pi0 V Pi0 V - ...)
 * (Pi0 is positive semidefinite for an independent-particle G, so W <= V).
 *   G_dev  : [ntau][n][n] device array (all tau points are used).
 *   W_dev  : [naux][naux] device array (output, caller-owned).
 * FP64 in every plan precision; 1 + V Pi0 is inverted by blocked Gauss-Jordan
 * elimination with partial pivoting (naux <= 9216, else THCSOX_EINVAL).  The
 * first call allocates 5 naux^2 doubles and the direct term's batch buffers
 * (kept by the plan).  THCSOX_ENONFINITE for a singular 1 + V Pi0.
 * Synchronises the plan's stream. */
int thcsox_static_screening(thcsox_plan_t p, const double* G_dev, double* W_dev);

/* Exchange self-energies with instantaneous screened lines of core W (e.g. from
 * thcsox_static_screening).  With Sigma[Va; Vc] the SOX sequence of
 * thcsox_sigma_sox with core Va on the line (pr|qs) (its U enters A) and core
 * Vc on the line (tu|vw) (its U enters C):
 *   THCSOX_SOSEX : Sigma = (Sigma[V; W] + Sigma[W; V]) / 2   (one line screened,
 *                  both placements; the symmetric-D path does not apply)
 *   THCSOX_G3W2  : Sigma = Sigma[W; W]                         (both lines screened)
 * for k in [k_begin, k_end), in the plan's precision (the U of W is built in
 * FP64 at every call and stored like the plan's U; the first call allocates
 * its planes).  G_dev, Sigma_dev: [ntau][n][n] device arrays (Sigma must not
 * alias G); W_dev: [naux][naux] device array, symmetric.  The energy is
 * thcsox_energy of the result.  Synchronises the plan's stream once (the U
 * build), then runs asynchronously. */
enum { THCSOX_SOSEX = 0, THCSOX_G3W2 = 1 };
int thcsox_sigma_screened(thcsox_plan_t p, const double* G_dev, const double* W_dev, int kind,
                          double* Sigma_dev, int k_begin, int k_end);

/* Back-projection alone (the last equation of the THC sequence):
 *     Sigma_tr = sum_PR X_tR Sig_RP X_rP       for k in [k_begin, k_end)
 *   Sigma_thc_dev[ntau][naux][naux] (read), Sigma_dev[ntau][n][n] (written).
 * Used to bring a self-energy given in the THC basis (e.g. a predicted one)
 * back to the orbital basis.  FP64, asynchronous. */
int thcsox_backproject(thcsox_plan_t p, const double* Sigma_thc_dev, double* Sigma_dev,
                       int k_begin, int k_end);

/* ---------------------------------------------------------------------------
 * IR basis and sparse sampling (computational-details section: the paper's loop
 * runs on the intermediate-representation grids of the references it cites,
 * at beta = 1000 and Lambda = 1e5).  Built on the host from the definition:
 * the singular value expansion of the fermionic kernel
 *     K(tau, omega) = exp(-tau omega) / (1 + exp(-beta omega)),
 *     tau in [0, beta], |omega| <= wmax, Lambda = beta wmax,
 * truncated at s_l / s_0 >= eps (L functions).  Sampling points: the L roots of
 * u_L in tau; the n >= 0 where the Matsubara transform of one of u_{L-3} .. u_L
 * changes sign, and n = 0, in frequency.
 *   thcsox_ir_create : eps in [1e-13, 1); Lambda <= 1e7.  Host-only (no HIP
 *       calls); about a second at Lambda = 1e5.  THCSOX_EINVAL for bad
 *       arguments or an eps finer than the FP64 discretisation resolves: the
 *       root count of u_L is checked, and a grid whose tau or frequency fit has
 *       a condition number above 1e4 is refused (a guard: the highest
 *       functions' transforms are at their noise level at low n).
 *   thcsox_ir_sizes  : ntau = L, nfreq.
 *   thcsox_ir_get    : copies (each pointer may be NULL) tau[ntau] ascending,
 *       freq_n[nfreq] ascending, Wf[2 nfreq][ntau] and Wb[ntau + 1][2 nfreq]
 *       (as thcsox_dyson_plan_sampled takes them), coef[ntau][ntau] (tau values
 *       -> coefficients) and sign[ntau] (u_l(beta - tau) = sign_l u_l(tau)) for
 *       thcsox_energy_basis, and the singular values sv[ntau] (tau, omega units).
 *   thcsox_ir_destroy: accepts NULL.
 * ------------------------------------------------------------------------- */
typedef struct thcsox_ir_s* thcsox_ir_t;
int thcsox_ir_create(thcsox_ir_t* out, double beta, double wmax, double eps);
int thcsox_ir_sizes(thcsox_ir_t g, int* ntau, int* nfreq);
int thcsox_ir_get(thcsox_ir_t g, double* tau, int* freq_n, double* Wf, double* Wb, double* coef,
                  double* sign, double* sv);
int thcsox_ir_destroy(thcsox_ir_t g);

/* Release a plan and all its device memory.  Accepts NULL. */
int thcsox_destroy(thcsox_plan_t p);

/* Message of the last failure on the calling thread ("" if none). */
const char* thcsox_last_error(void);

/* Sizes and per-tau work of a plan, for roofline accounting. */
typedef struct {
  int n, naux, ntau, precision;
  int tau_batch;              /* tau points processed per batch */
  size_t bytes;               /* device bytes owned by the plan */
  double mac_per_tau;         /* algorithmic multiply-adds per tau point:
                                 2 naux^2 n^2 + naux n^3 + 2 naux^2 n + 3 naux n^2 */
  double fused_mac_per_tau;   /* of which in the fused B/C/D kernel: 2 naux^2 n^2 */
  double fused_bytes_per_tau; /* compulsory HBM bytes of the fused kernel per tau:
                                 U and A once each, plus the projected G */
  int vsplit;                 /* v ranges of the fused kernel (partial D tiles per tau) */
  int vrange;                 /* longest v range */
  int partial_f32;            /* 1: partial D tiles are FP32 (each holds one FP32
                                 partial sum), 0: FP64 */
} thcsox_plan_info_t;
int thcsox_plan_info(thcsox_plan_t p, thcsox_plan_info_t* info);

/* ---------------------------------------------------------------------------
 * One self-consistency step in FP64 (Sec. "Definitions": Eq. Dyson in an
 * orthonormal basis, and the density matrix gamma_pq = -G_qp(0^-), taken as
 * gamma = -G(beta^-)):
 *   Sigma(tau) on the Chebyshev-root grid -> Chebyshev interpolation ->
 *   Sigma(i w_n), w_n = (2n+1) pi / beta, n = 0 .. n_matsubara-1 ->
 *   G(i w_n) = [(i w_n + mu) 1 - F - Sigma(i w_n)]^-1 ->
 *   least-squares Chebyshev fit over the kept frequencies -> G(tau_k), gamma.
 * The grid must be the m roots of T_m mapped to [0, beta] (ascending).
 * ------------------------------------------------------------------------- */
typedef struct thcsox_dyson_s* thcsox_dyson_t;

/* F_dev[n][n]: one-body operator (copied).  mu: chemical potential (fixed).
 * Needs 2 n_matsubara >= ntau and n <= 9216 (the inversion keeps an n x b
 * panel of each frequency's matrix in LDS, b = 8 for n <= 1152).  Device
 * memory: about n_matsubara n^2 x 48 bytes.  Synchronises the stream. */
int thcsox_dyson_plan(thcsox_dyson_t* out, int n, int ntau, int n_matsubara, double beta,
                      double mu, const double* tau_host, const double* F_dev, void* hip_stream);

/* Sigma_dev[ntau][n][n] (read) -> G_dev[ntau][n][n] and gamma_dev[n][n] (written;
 * gamma_dev may be NULL).  The inversion is blocked in-place Gauss-Jordan
 * elimination with partial pivoting.  Synchronises the stream;
 * THCSOX_ENONFINITE if a pivot is zero or not finite (singular matrix). */
int thcsox_dyson_step(thcsox_dyson_t d, const double* Sigma_dev, double* G_dev,
                      double* gamma_dev);

/* The same step with the chemical potential chosen so that the electron number
 * is conserved (size-consistency appendix, "optimized chemical potential";
 * Sec. "Definitions": the Dyson solution "with the update of the chemical
 * potential"): mu such that Tr gamma(mu) = nelec to within tol, where gamma(mu)
 * comes from the Dyson solve at mu (Sigma(i w) is formed once).  Search: from
 * *mu_io, steps of 0.1 Ha doubled until N(mu) - nelec changes sign, then the
 * Illinois variant of regula falsi; at most 80 Dyson solves.  On success *mu_io
 * is the chemical potential used (also kept by the plan for later
 * thcsox_dyson_step calls), G_dev / gamma_dev are as for thcsox_dyson_step at
 * that mu, and *evals_out (may be NULL) is the number of Dyson solves.
 * THCSOX_EINVAL unless 0 <= nelec <= n and tol > 0; THCSOX_ENONFINITE if a
 * matrix is singular or no bracket / no convergence within the limit.
 * Synchronises the stream once per Dyson solve. */
int thcsox_dyson_step_mu(thcsox_dyson_t d, const double* Sigma_dev, double nelec, double tol,
                         double* mu_io, double* G_dev, double* gamma_dev, int* evals_out);

/* A Dyson plan on caller-given sampling grids (e.g. the IR grids of
 * thcsox_ir_create) instead of the Chebyshev grid: ntau tau points, and nfreq
 * fermionic frequencies w_j = (2 freq_n[j] + 1) pi / beta, freq_n ascending,
 * >= 0 (the negative ones are the complex conjugates for real G(tau)).
 *   Wf_host [2 nfreq][ntau]   : [Re; Im] F(i w_j) = Wf F(tau)
 *   Wb_host [ntau + 1][2 nfreq]: F(tau_k) (rows 0..ntau-1) and F(beta^-) (last
 *                                row) from [Re; Im] F(i w_j)
 * Both are copied.  Steps, the mu search and the energies are then as for
 * thcsox_dyson_plan (gamma = -G(beta^-) from the last row of Wb).  THCSOX_EINVAL
 * for 2 nfreq < ntau, unsorted or negative freq_n, or non-finite tables. */
int thcsox_dyson_plan_sampled(thcsox_dyson_t* out, int n, int ntau, int nfreq, double beta,
                              double mu, const int* freq_n_host, const double* Wf_host,
                              const double* Wb_host, const double* F_dev, void* hip_stream);

/* E1 = Tr[F gamma] = sum_pq F_pq gamma_qp in FP64 (host scalar). */
int thcsox_dyson_onebody(thcsox_dyson_t d, const double* gamma_dev, double* E1_host);

int thcsox_dyson_destroy(thcsox_dyson_t d);

/* ---------------------------------------------------------------------------
 * Convergence aids for the self-consistency loop on device arrays of doubles
 * (the paper's loop uses damping and DIIS-type linear combinations of
 * self-energies; this is Pulay DIIS on the residual Sigma_out - Sigma_in, not
 * the paper's frequency-dependent commutator variant).
 * ------------------------------------------------------------------------- */

/* Damping: sigma_io = alpha sigma_io + (1 - alpha) sigma_out, len doubles,
 * asynchronous on hip_stream (NULL: the default stream). */
int thcsox_mix(int64_t len, double alpha, const double* sigma_out, double* sigma_io,
               void* hip_stream);

typedef struct thcsox_diis_s* thcsox_diis_t;

/* History of the last `depth` (Sigma_in, Sigma_out - Sigma_in) pairs, len doubles
 * each, kept on the device (2 depth len doubles); depth >= 1. */
int thcsox_diis_create(thcsox_diis_t* out, int64_t len, int depth, void* hip_stream);

/* Adds (sigma_in, sigma_out) to the history (dropping the oldest beyond depth)
 * and writes sigma_next = sum_i c_i Sigma_out_i with c minimising
 * |sum_i c_i r_i|^2 under sum_i c_i = 1 (r_i the residuals; dot products in FP64
 * on the device, the bordered (k+1) x (k+1) system solved on the host).  If that
 * system is singular the oldest entries are dropped until it is not.
 * sigma_next may alias sigma_in but not sigma_out.  Synchronises the stream.
 * *n_used_out (may be NULL): the number of history entries combined. */
int thcsox_diis_step(thcsox_diis_t d, const double* sigma_in, const double* sigma_out,
                     double* sigma_next, int* n_used_out);

/* Commutator DIIS (the paper's loop uses a frequency-dependent commutator DIIS
 * from the algorithms paper it cites, Sec. "Computational details"; that
 * paper's formula is not printed, reading used): with G_i = Dyson(Sigma_in_i),
 * G_i(i w) commutes with the matrix it inverts, so the error of iteration i is
 *     e_i(i w_n) = [G_i(i w_n), F + Sigma_out_i(i w_n)]
 *                = G_i D_i - D_i G_i,   D_i = Sigma_out_i(i w_n) - Sigma_in_i(i w_n)
 * on the plan's frequencies (n >= 0).  thcsox_dyson_commutator writes e for
 * the G(i w) of the plan's last Dyson step (which must have been taken with
 * Sigma_in_dev): e_dev [2][nfreq][n][n] (real parts, then imaginary parts),
 * FP64 matrix cores, asynchronous.  The first call allocates 2 nfreq n^2
 * doubles (kept by the plan).  THCSOX_EINVAL before the plan's first step. */
int thcsox_dyson_commutator(thcsox_dyson_t d, const double* Sigma_in_dev,
                            const double* Sigma_out_dev, double* e_dev);

/* A DIIS history whose residuals the caller supplies (len_res doubles each,
 * e.g. the commutator of thcsox_dyson_commutator, len_res = 2 nfreq n^2) next
 * to the extrapolated vectors (len doubles, Sigma_out): thcsox_diis_step_res
 * adds (residual, sigma_out) and writes sigma_next = sum_i c_i Sigma_out_i with
 * c minimising |sum_i c_i e_i|^2 under sum_i c_i = 1 (B_ij = <e_i, e_j> over all
 * real and imaginary parts, i.e. Re sum_n Tr[e_i^H e_j]), dropping the oldest
 * entries while the bordered system is singular.  sigma_next may alias the
 * inputs.  Synchronises the stream.  A history made by thcsox_diis_create
 * refuses thcsox_diis_step_res and vice versa (THCSOX_EINVAL). */
int thcsox_diis_create_res(thcsox_diis_t* out, int64_t len, int64_t len_res, int depth,
                           void* hip_stream);
int thcsox_diis_step_res(thcsox_diis_t d, const double* residual, const double* sigma_out,
                         double* sigma_next, int* n_used_out);

int thcsox_diis_destroy(thcsox_diis_t d);

/* ---------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method; it only proposes a
 * starting self-energy that the plain SOX loop then corrects).  A residual MLP
 * on the tau-profile of one THC pair (m inputs, m outputs, two hidden layers
 * of width H, silu, FP32 weights and matrix cores):
 *     y = x + W3 silu(W2 silu(W1 x + b1) + b2) + b3
 * params: one packed FP32 array W1[H][m], b1[H], W2[H][H], b2[H], W3[m][H], b3[m].
 * x, y, target: [batch][m] FP32 device arrays.  Loss: mean squared error.
 * ------------------------------------------------------------------------- */
typedef struct thcsox_mlp_s* thcsox_mlp_t;
int thcsox_mlp_create(thcsox_mlp_t* out, int m, int hidden, int max_batch,
                      const float* params_host, void* hip_stream);
/* Inference for any batch size (processed max_batch rows at a time); asynchronous. */
int thcsox_mlp_forward(thcsox_mlp_t q, const float* x_dev, float* y_dev, int batch);
/* Inference with bf16 weights, for any batch size, asynchronous: the network's
 * parameters rounded to bf16 (nearest, ties to even; re-rounded after training
 * steps), each layer's input (x, h1, h2) rounded to bf16, bf16 matrix cores
 * with FP32 accumulation, bias, silu and the residual add on the exact FP32 x
 * in FP32.  One fused kernel per 64 rows keeps the hidden activations in LDS
 * (no max_batch limit, no activation buffers).  Needs m in {32, 64} and H in
 * {128, 256, 512} (THCSOX_EINVAL otherwise); batch 0 does nothing (x and y
 * may then be NULL); the first call allocates the bf16 parameter copy.  y may
 * not alias x. */
int thcsox_mlp_forward_bf16(thcsox_mlp_t q, const float* x_dev, float* y_dev, int64_t batch);
/* Loss and its gradient with respect to every parameter (packed like params);
 * batch <= max_batch.  grads_host may be NULL.  Synchronises. */
int thcsox_mlp_gradients(thcsox_mlp_t q, const float* x_dev, const float* target_dev, int batch,
                         float* grads_host, double* loss_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * gradient of one batch; loss_host (may be NULL) receives the batch loss
 * before the step (then the call synchronises). */
int thcsox_mlp_train_step(thcsox_mlp_t q, const float* x_dev, const float* target_dev, int batch,
                          float lr, double* loss_host);
int thcsox_mlp_params(thcsox_mlp_t q, float* params_host);
int thcsox_mlp_destroy(thcsox_mlp_t q);

/* Network inputs and outputs in the THC basis.  S is a THC-basis self-energy
 * [m][naux][naux] (FP64, device); a "pair" is the flat index R*naux + P.
 *   thcsox_pair_scale  : scale[p] = max_k |S[k][p]| (1 if zero), the pair's
 *                        largest magnitude over tau, FP64 [naux^2].
 *   thcsox_pair_gather : x[b][k] = S[k][pairs[b]] / scale[pairs[b]] (pairs NULL:
 *                        all naux^2 pairs in order), FP32 [npairs][m].
 *   thcsox_pair_scatter: S[k][p] = y[p][k] * scale[p] for all naux^2 pairs.
 * All asynchronous on hip_stream. */
int thcsox_pair_scale(int m, int naux, const double* S_dev, double* scale_dev, void* hip_stream);
int thcsox_pair_gather(int m, int naux, const double* S_dev, const double* scale_dev,
                       const long long* pairs_dev, long long npairs, float* x_dev,
                       void* hip_stream);
int thcsox_pair_scatter(int m, int naux, const float* y_dev, const double* scale_dev,
                        double* S_dev, void* hip_stream);

/* Optional stage timing with HIP events recorded on the plan's stream around
 * each stage of every tau point (negligible overhead).  Stages:
 *   THCSOX_STAGE_PROJECT : projections G_Rq, G_wP, G(-tau) and their scaling/splits
 *   THCSOX_STAGE_A       : A_Pqv = sum_s U_Pqs G_sv(-tau) (and its split)
 *   THCSOX_STAGE_FUSED   : the fused B/C/D kernel
 *   THCSOX_STAGE_BACK    : reduction of D, Sig_RP and the back-projection
 * thcsox_profile(p, 1) starts recording (and clears what was recorded);
 * thcsox_stage_times synchronises the stream and returns, per stage, the total
 * milliseconds and the number of timed launches since the last read, then clears. */
enum {
  THCSOX_STAGE_PROJECT = 0,
  THCSOX_STAGE_A = 1,
  THCSOX_STAGE_FUSED = 2,
  THCSOX_STAGE_BACK = 3,
  THCSOX_NSTAGES = 4
};
int thcsox_profile(thcsox_plan_t p, int enable);
int thcsox_stage_times(thcsox_plan_t p, double* ms /*[THCSOX_NSTAGES]*/,
                       int* launches /*[THCSOX_NSTAGES]*/);

#ifdef __cplusplus
}
#endif
#endif /* THCSOX_H */
