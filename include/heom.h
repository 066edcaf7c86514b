/*
 * heom.h -- C ABI of the MI355X HEOM library (matrix-free HEOM Liouvillian
 * apply, RK4 propagation, stationary state, spectra, batched solves and a
 * learned block preconditioner), after arXiv 2306.07522.
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Complex numbers are interleaved (re, im).  Host matrices are d x d,
 *    row-major, complex double.
 *  - An ADO vector is [N][d][d] complex (row-major blocks, ADO index major);
 *    with R right-hand sides it is [N][d][d][R] (R innermost).  FP64 vectors
 *    hold double pairs, FP32 vectors float pairs.  ADO 0 is the reduced
 *    density operator.
 *  - Fermionic ADOs are antisymmetric in their exponent indices: the stored
 *    ADO of an exponent set S is rho_{[s_n .. s_1]} with s_n > ... > s_1 in
 *    the exponent numbering below.  Bosonic ADOs are symmetric and are
 *    stored once per multiset, unnormalised (no sqrt(n!) factors).
 *  - Exponent numbering: bosonic exponents in bath-record order, then in
 *    list order; fermionic exponents in bath-record order, then h, then
 *    nu = +1 before nu = -1 (index = base + 2h + (nu == -1)).
 *  - Device pointers are HIP device memory owned by the caller; `stream`
 *    is a hipStream_t (NULL = default stream).  Host pointers are read
 *    during the call only.
 *  - No exception crosses the ABI.  Every entry point returns a status;
 *    on error the outputs are unspecified and heom_last_error() returns a
 *    thread-local message.
 *  - A handle is immutable after build and may be used from several
 *    host threads and streams at once provided each call has its own
 *    workspace.  Its device tables are uploaded by the first call that
 *    needs them, once, under a lock held by the handle.  The exceptions are
 *    heom_hierarchy_set_lindblad and heom_free, which change or release the
 *    handle and must not overlap any other call on it.
 */
#ifndef HEOM_H
#define HEOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t heom_status;
enum {
  HEOM_OK = 0,
  HEOM_ERR_ARG = 1,           /* invalid argument                       */
  HEOM_ERR_ALLOC = 2,         /* host or device allocation failed        */
  HEOM_ERR_HIP = 3,           /* a HIP runtime call failed               */
  HEOM_ERR_NOT_CONVERGED = 4, /* iterative solver hit its limit          */
  HEOM_ERR_SINGULAR = 5,      /* breakdown / zero pivot                  */
  HEOM_ERR_UNSUPPORTED = 6,   /* size or feature outside what is built   */
  HEOM_ERR_NAN = 7            /* non-finite value detected               */
};

enum { HEOM_FP64 = 0, HEOM_FP32 = 1 };
enum { HEOM_BOSON = 0, HEOM_FERMION = 1 };
/* bosonic exponent type u (eq:C_beta_RI): real part, imaginary part, or
 * both at once when chi is real */
enum { HEOM_U_R = 0, HEOM_U_I = 1, HEOM_U_RI = 2 };
enum { HEOM_PADE = 0, HEOM_MATSUBARA = 1 };

typedef struct heom_hier heom_hier; /* opaque hierarchy + device tables  */
typedef struct heom_nn heom_nn;     /* opaque learned preconditioner     */

/* ------------------------------------------------------------------------
 * Exponents (Methods: Lorentzian fermionic and Drude-Lorentz bosonic
 * correlation functions; eq:C_f_exp, eq:C_b_exp)
 * ---------------------------------------------------------------------- */

/* [N-1/N] Pade (method HEOM_PADE) or Matsubara (HEOM_MATSUBARA)
 * parameters of the Fermi (kind HEOM_FERMION) or Bose (HEOM_BOSON)
 * function: n_F(x) ~ 1/2 - sum 2 kappa x/(x^2 + zeta^2),
 * n_B(x) ~ 1/x - 1/2 + sum 2 kappa x/(x^2 + zeta^2).  kappa, zeta: host
 * arrays of n doubles, zeta ascending.  n in [0, 64]. */
heom_status heom_pade_params(int32_t kind, int32_t method, int32_t n, double *kappa, double *zeta);

/* Lorentzian lead J = Gamma W^2 / ((w - mu)^2 + W^2) at temperature T with
 * n_exp terms (h = 1 the J pole, h >= 2 distribution poles).  Outputs are
 * host complex arrays of n_exp: eta and gamma for nu = +1 and nu = -1.
 *   eta_1 = (Gamma W / 2) n_F(i W / T), gamma^nu_1 = W - nu i mu,
 *   eta_h = -i kappa T Gamma W^2 / (W^2 - (zeta T)^2),
 *   gamma^nu_h = zeta T - nu i mu. */
heom_status heom_exponents_lorentz(double Gamma, double W, double mu, double T, int32_t n_exp,
                                   int32_t method, double *eta_p, double *gam_p, double *eta_m,
                                   double *gam_m);

/* Drude-Lorentz bath J = 4 lam gamma w / (w^2 + gamma^2) (with the 1/2pi
 * of eq:C_b) at temperature T, n_exp terms, all with real chi ("RI"):
 *   xi_1 = lam gamma (cot(gamma / 2T) - i), chi_1 = gamma,
 *   xi_l = 4 kappa lam gamma T (zeta T) / ((zeta T)^2 - gamma^2), chi_l = zeta T.
 * xi, chi: host complex arrays of n_exp. */
heom_status heom_exponents_drude_lorentz(double lam, double gamma, double T, int32_t n_exp,
                                         int32_t method, double *xi, double *chi);

/* ------------------------------------------------------------------------
 * Hierarchy (eq:HEOM, the multi-index paragraph and the truncation rules)
 * ---------------------------------------------------------------------- */

/* One bath = one coupling operator and its exponents (Fig. 1b). */
typedef struct {
  int32_t kind;           /* HEOM_BOSON (V Hermitian) or HEOM_FERMION (d)   */
  const double *op;       /* d x d complex: V, or the annihilation op d     */
  int32_t n_exp;          /* boson: number of exponents; fermion: number of h */
  /* boson */
  const int32_t *u_type;  /* n_exp of HEOM_U_R / HEOM_U_I / HEOM_U_RI        */
  const double *xi;       /* n_exp complex                                   */
  const double *chi;      /* n_exp complex                                   */
  /* fermion: h-paired lists for nu = +1 and nu = -1 */
  const double *eta_p, *gam_p, *eta_m, *gam_m; /* n_exp complex each        */
} heom_bath;

typedef struct {
  int64_t n_ado;          /* N                                               */
  int32_t d;
  int32_t n_bos_exp;      /* K_b                                             */
  int32_t n_ferm_exp;     /* K_f                                             */
  int32_t m_max, n_max;   /* effective truncation tiers                      */
  int32_t parity;         /* +1 even, -1 odd                                 */
  int32_t n_ops;          /* distinct operators (H, V's, d and d^dagger's)   */
  int64_t n_edges;        /* tier-coupling terms (neighbour table entries)   */
  int64_t n_leaf;         /* ADOs with no higher-tier neighbour              */
  int32_t n_tiers;        /* number of (m + n) tiers                         */
  int64_t tier_offset[34];/* first ADO of each tier, tier_offset[n_tiers] = N */
  int64_t table_bytes;    /* device bytes of the neighbour/decay tables      */
  int64_t vector_bytes_fp64; /* N d^2 * 16                                   */
} heom_info;

/* Build the hierarchy of ADOs for system Hamiltonian H (d x d Hermitian)
 * coupled to n_baths baths, truncated at bosonic tier m_max and fermionic
 * tier n_max, in parity sector `parity` (+1 even, -1 odd; eq:HEOM's p).
 * Host-side only: device tables are uploaded on the first device call.
 * parity_op: optional d x d fermionic parity operator; when given, H and
 * every bosonic V must commute with it and every fermionic d anticommute
 * (HEOM_ERR_ARG otherwise).  Checks: H and V Hermitian (1e-12 relative),
 * K_f <= 64, d <= 64, N < 2^31.  *out is released with heom_free. */
heom_status heom_build_hierarchy(int32_t d, const double *H, int32_t n_baths, const heom_bath *baths,
                                 int32_t m_max, int32_t n_max, int32_t parity,
                                 const double *parity_op, heom_hier **out);
/* As heom_build_hierarchy, leaving out the ADOs of low importance (the
 * truncation paragraph after eq:HEOM, eq:importance): an ADO with bosonic
 * level m > 1 or fermionic level n > 1 is dropped when
 *   |prod_r xi_{j_r} / (Re chi_{j_r} sum_{x<=r} Re chi_{j_x})| *
 *   |prod_w eta_{q_w} / (Re gamma_{q_w} sum_{x<=w} Re gamma_{q_x})|
 * is below importance_threshold (>= 0; 0 keeps every ADO).  The products
 * run over the ADO's exponents in list order: bosonic exponents in bath
 * order, fermionic ones per bath with the nu = +1 terms h = 1.. first and
 * then the nu = -1 terms (the order that reproduces the counts of Table 3).
 * Terms of eq:HEOM that would reach a dropped ADO are left out, as for ADOs
 * beyond the tier cutoff. */
heom_status heom_build_hierarchy_pruned(int32_t d, const double *H, int32_t n_baths, const heom_bath *baths,
                                        int32_t m_max, int32_t n_max, int32_t parity, const double *parity_op,
                                        double importance_threshold, heom_hier **out);
/* Lindbladian add-on (eq:Lindbladian and the construction paragraph around
 * it): every ADO of h additionally evolves under
 *   sum_k J(F_k)[X],  J(F)[X] = F X F^dagger - 1/2 {F^dagger F, X},
 * which describes extra, Markovian environments without adding ADOs.  F:
 * host, n_ops matrices of d x d complex (row-major, interleaved re/im),
 * copied; rates go into the operators (F = sqrt(rate) L).  n_ops = 0 removes
 * them.  With a parity operator given at build, each F must commute with
 * it.  Every apply (heom_apply*, heom_propagate, heom_steady, heom_spectrum)
 * includes the term; the preconditioners ignore it.  The device tables are
 * uploaded again on the next use.  Errors: HEOM_ERR_ARG (NULL, non-finite,
 * parity-odd F), HEOM_ERR_UNSUPPORTED (d > 32).  A hierarchy with a
 * Lindbladian cannot join a batch. */
heom_status heom_hierarchy_set_lindblad(heom_hier *h, int32_t n_ops, const double *F);
void heom_free(heom_hier *h);
heom_status heom_hierarchy_info(const heom_hier *h, heom_info *out);

/* Hierarchy dictionary (Fig. 1e): the multi-index of every ADO.
 * bos_occ: host int32 [N][K_b] occupation of each bosonic exponent (may be
 * NULL); ferm_mask: host uint64 [N] bit k set when fermionic exponent k is
 * present (may be NULL); level: host int32 [N][2] = (m, n) (may be NULL). */
heom_status heom_hierarchy_ados(const heom_hier *h, int32_t *bos_occ, uint64_t *ferm_mask, int32_t *level);

/* Inverse lookup: the index of the ADO whose bosonic occupations are
 * bos_occ[K_b] and whose fermionic exponents are ferm_ids[n_f] in the
 * given order; *sign receives the permutation sign that relates the given
 * order to the stored one (rho_given = sign * rho_stored).  *idx = -1 when
 * the ADO is outside the hierarchy. */
heom_status heom_ado_index(const heom_hier *h, const int32_t *bos_occ, const int32_t *ferm_ids,
                           int32_t n_f, int64_t *idx, int32_t *sign);

/* Host copy of the diagonal decay c_a = sum_k n_k chi_k + sum_{q in a} gamma_q
 * (complex [N]) and of the neighbour table in CSR form: row_ptr [N+1],
 * col [E] (neighbour ADO), kind [E] (0 bos up, 1 bos down, 2 ferm up,
 * 3 ferm down), exp [E] (exponent index), mult [E] (bosonic multiplicity or
 * fermionic reorder sign).  Any pointer may be NULL. */
heom_status heom_hierarchy_tables(const heom_hier *h, double *decay, int64_t *row_ptr, int32_t *col,
                                  int32_t *kind, int32_t *exp, int32_t *mult);

/* Uploads the hierarchy's device tables and launch plans to the current
 * device now, instead of on the first device call.  Allocates device memory
 * (held by the handle until heom_free); call it before capturing work that
 * uses the handle into a hipGraph, since a capture cannot allocate.  Safe to
 * call from several threads on one handle: the upload runs once.
 * HEOM_ERR_ARG if the tables already live on another device. */
heom_status heom_prepare(heom_hier *h);

/* ------------------------------------------------------------------------
 * Liouvillian apply (eq:HEOM; the HEOMLS M acting on the ADO vector)
 * ---------------------------------------------------------------------- */

/* y = (M + shift I) x for n_rhs right-hand sides ([N][d][d][R] vectors).
 * shift: host pointer to one complex number applied to every right-hand
 * side, or NULL for zero.  precision HEOM_FP64 / HEOM_FP32 selects the
 * element type of x and y.  x and y must not overlap.  Device tables are
 * uploaded on the first call (this first call allocates).  Asynchronous on
 * `stream`. */
heom_status heom_apply(heom_hier *h, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                       const double *shift, void *stream);

/* As heom_apply, with one shift per right-hand side: column r gets
 * shifts_dev[r], a device array of n_rhs complex numbers of the same
 * precision as x and y. */
heom_status heom_apply_shifted(heom_hier *h, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                               const void *shifts_dev, void *stream);

/* y = B x with B the stationary-state operator: M (even parity) with the
 * equation of element (0,0) of ADO 0 replaced by the trace condition,
 * (B x)_{0,00} = sum_i (x_0)_{ii} (the system heom_steady solves with
 * right-hand side e_0).  Same conventions as heom_apply, one right-hand
 * side. */
heom_status heom_apply_steady_operator(heom_hier *h, int32_t precision, const void *x_dev, void *y_dev,
                                       void *stream);

/* Launch plans of the apply (eq:HEOM's terms are the same in every plan;
 * only the order of the floating-point additions differs).
 *  HEOM_PLAN_AUTO  the default of every other entry point: the pull plan,
 *                  as HEOM_PLAN_PULL_MFMA when d = 16, one right-hand side
 *                  and H has at least 8 (FP64) or 12 (FP32) off-diagonal
 *                  entries in some row or column (the measured cut-over);
 *  HEOM_PLAN_PULL  one launch: every ADO gathers all its neighbour blocks;
 *  HEOM_PLAN_SLAB  three launches: the lower tiers and the top tier's own
 *                  rows, then two launches over label slabs of the top two
 *                  fermionic tiers in which the parents' up-terms are summed
 *                  while each top-tier block passes through LDS once per
 *                  launch.  Fewer bytes from memory, but slower than the pull
 *                  plan where measured (two-orbital model, d = 16).  Built for
 *                  purely fermionic hierarchies without pruning, n_max >= 3,
 *                  d = 8 or 16, one right-hand side; HEOM_ERR_UNSUPPORTED
 *                  otherwise.
 *  HEOM_PLAN_PULL_MFMA  the pull plan with the H terms of every ADO's own
 *                  block (-i[H, rho_a] without H's diagonal) computed as
 *                  dense 16 x 16 complex products on the matrix cores
 *                  (16 x 16 x 4 MFMA, FP64 or FP32 as the vectors) instead
 *                  of the sparse gathers.  d = 16, one right-hand side;
 *                  HEOM_ERR_UNSUPPORTED otherwise. */
enum { HEOM_PLAN_AUTO = 0, HEOM_PLAN_PULL = 1, HEOM_PLAN_SLAB = 2, HEOM_PLAN_PULL_MFMA = 3 };

/* Layout of the slab plan, computed on the host without touching the
 * device (the plan itself is uploaded with the other tables on first use):
 * per launch (0 = A, 1 = B) the workgroup count (empty XCD slots included),
 * the child entries (a child counts once per workgroup that reads it), the
 * most parents one workgroup holds, and the estimated cost per XCD in block
 * reads.  built = 0 when the hierarchy has no slab plan.  The build checks
 * that every ADO's row (self term and every neighbour term) is scheduled
 * exactly once and fails with HEOM_ERR_ARG otherwise. */
typedef struct {
  int32_t built;
  int32_t max_vertices[2];
  int64_t children, parents;
  int64_t jobs[2], entries[2], cost[2];
  int64_t xcd_cost[2][8];
} heom_slab_stats;
heom_status heom_slab_plan_stats(const heom_hier *h, heom_slab_stats *out);

/* heom_apply with an explicit launch plan (HEOM_PLAN_*); same arguments,
 * same result up to rounding order. */
heom_status heom_apply_plan(heom_hier *h, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                            const double *shift, int32_t plan, void *stream);

/* Apply with the top tier split into `n_chunks` column blocks (one launch
 * per block plus one for the lower tiers) so that each block's neighbour
 * reads stay cache-resident.  Same result as heom_apply up to rounding
 * order.  n_chunks <= 0 picks the library default. */
heom_status heom_apply_tiled(heom_hier *h, int32_t precision, const void *x_dev, void *y_dev,
                             int32_t n_rhs, const double *shift, int32_t n_chunks, void *stream);

/* ------------------------------------------------------------------------
 * Time propagation (Fig. 1d; fixed-step classical RK4)
 * ---------------------------------------------------------------------- */

/* Integrate dx/dt = M x from x(0) (in x_dev) for n_steps steps of dt; on
 * return x_dev holds x(n_steps dt).  If rho0_traj_dev is not NULL it
 * receives the reduced density operator (ADO 0, d*d complex of the given
 * precision) after every save_every steps: n_steps / save_every entries.
 * Workspace: heom_workspace_size(HEOM_OP_PROPAGATE).  graph_steps > 0
 * captures that many steps in a hipGraph and replays it.  Hierarchies of at
 * most 1024 complex elements (N d^2) run many whole steps per launch in one
 * workgroup instead (graph_steps is then ignored). */
heom_status heom_propagate(heom_hier *h, int32_t precision, void *x_dev, double dt, int64_t n_steps,
                           int64_t save_every, void *rho0_traj_dev, int32_t graph_steps, void *ws,
                           size_t ws_bytes, void *stream);

/* Time-dependent system Hamiltonian H_s(t) = H + sum_k f_k(t) V_k in RK4
 * (the paper allows H_s(t) in the dynamics; "Package architecture").  As
 * heom_propagate (same x_dev, save_every, traj_dev and workspace, whose size
 * is heom_workspace_size(HEOM_OP_PROPAGATE)), starting at time t0; every
 * RK4 stage adds -i sum_k f_k(t_stage) [V_k, X] to each ADO, with the stage
 * times t, t + dt/2, t + dt/2, t + dt.  V: host, n_drive (1..8) Hermitian
 * d x d complex matrices (row-major, interleaved), copied; with a parity
 * operator given at build each V_k must commute with it.  f(t, coef, ctx)
 * writes the n_drive real coefficients at time t; it is called on the host,
 * four times per step, before the stage's kernels are enqueued.  Steps run
 * eagerly (no graph; hierarchies of any size take the general kernels).
 * Synchronises the stream before returning.  Errors: HEOM_ERR_ARG (bad
 * arguments, non-Hermitian or parity-odd V, workspace too small),
 * HEOM_ERR_NAN (a non-finite coefficient), HEOM_ERR_UNSUPPORTED (d > 32). */
typedef void (*heom_drive_fn)(double t, double *coef, void *ctx);
heom_status heom_propagate_driven(heom_hier *h, int32_t precision, void *x_dev, double t0, double dt,
                                  int64_t n_steps, int64_t save_every, void *rho0_traj_dev, int32_t n_drive,
                                  const double *V, heom_drive_fn f, void *ctx, void *ws, size_t ws_bytes,
                                  void *stream);

/* ------------------------------------------------------------------------
 * Linear solves (stationary state and spectra)
 * ---------------------------------------------------------------------- */
enum { HEOM_OP_PROPAGATE = 0, HEOM_OP_STEADY = 1, HEOM_OP_SPECTRUM = 2 };
/* Preconditioners (right): none; Jacobi, the inverse diagonal of the system;
 * the learned network (HEOM_PREC_NN, see below); SCALED, division by the
 * modulus of the diagonal, a positive scaling that leaves the orientation of
 * the operator's left-half-plane spectrum alone (Jacobi's complex phases
 * rotate parts of it around the origin, which can slow restarted GMRES). */
/* HEOM_PREC_BLOCK: per ADO, the exact inverse of the ADO's own terms of
 * eq:HEOM, -(c_a - z) X - i[H, X], applied in the eigenbasis of H
 * (H = U diag(E) U^H, so X -> U ((U^H X U) / D) U^H with
 * D_ij = -(c_a - z) - i(E_i - E_j)).  Entries with |D_ij| below the slowest
 * bath decay rate (min Re chi, Re gamma) are divided by minus that rate
 * instead.  It keeps the whole coherent part of each ADO's dynamics, where
 * Jacobi keeps only the diagonal of H; with weak baths this is the part that
 * stalls restarted GMRES.  Requires d <= 32 (HEOM_ERR_UNSUPPORTED otherwise). */
enum { HEOM_PREC_NONE = 0, HEOM_PREC_JACOBI = 1, HEOM_PREC_NN = 2, HEOM_PREC_SCALED = 3, HEOM_PREC_BLOCK = 4 };
/* HEOM_SOLVE_SHIFTED (heom_spectrum only, precond HEOM_PREC_NONE): all
 * frequencies share one Krylov space of the unshifted operator (restarted
 * full orthogonalisation, whose residuals stay parallel across shifts);
 * only the trace readout of each solution is accumulated, so memory does not
 * grow with the number of frequencies.  The report's true residual is the
 * largest of the FOM residual estimates and of the true residuals of three
 * probe frequencies (first, middle, last), measured with the plain apply. */
enum { HEOM_SOLVE_FP64 = 0, HEOM_SOLVE_FP32_IR = 1, HEOM_SOLVE_SHIFTED = 2 };

typedef struct {
  int32_t restart;        /* GMRES restart length m (default 30)              */
  int32_t max_iter;       /* total inner iterations (default 3000)            */
  double tol;             /* relative true residual ||b - A x|| / ||b||       */
  int32_t precond;        /* HEOM_PREC_*                                      */
  int32_t mode;           /* HEOM_SOLVE_FP64, HEOM_SOLVE_FP32_IR, or (spectra)
                             HEOM_SOLVE_SHIFTED                               */
  double inner_tol;       /* FP32 inner tolerance for IR (default 1e-5)       */
  int32_t max_refine;     /* IR outer steps (default 20)                      */
  int32_t rhs_chunk;      /* spectra: frequencies per multi-RHS solve; 0 =
                             automatic (heom_spectrum_chunk)               */
  const heom_nn *nn;      /* learned preconditioner for HEOM_PREC_NN          */
  int32_t fallback;       /* 1: on NN failure (NaN, max_iter, or an FP64
                             restart cycle that cuts the true residual by
                             less than 10%) solve again with Jacobi, with a
                             fresh max_iter, from the network's iterate if
                             its residual is <= 0.1, else from zero; the
                             report sums both attempts                     */
  int32_t use_x0;         /* 1: x_dev holds the initial guess                 */
  int32_t deflate;        /* 0 = plain restarts; k > 0 = deflated restarts,
                             so that slow modes of the operator stay in
                             the Krylov space.  heom_steady: GMRES-DR
                             (Morgan 2002), each restart keeps the k
                             harmonic Ritz vectors of smallest harmonic
                             Ritz value and the residual.  heom_spectrum
                             in HEOM_SOLVE_SHIFTED mode: thick
                             (Krylov-Schur) restarts of the multi-shift
                             FOM, each full cycle keeps the Schur vectors
                             of the k Ritz values of M nearest the negated
                             unconverged shifts -i(+-omega) and the common
                             residual direction.  1 <= k <= 31,
                             k <= restart - 2, precond not HEOM_PREC_NN;
                             other entry points and modes reject k != 0 */
} heom_solver_opts;

typedef struct {
  int32_t status;         /* HEOM_OK or HEOM_ERR_NOT_CONVERGED / _NAN          */
  int32_t iterations;     /* inner iterations (summed over RHS chunks)         */
  int32_t restarts;
  int32_t refinements;    /* IR outer steps                                    */
  int32_t fell_back;      /* 1 when the NN preconditioner was abandoned        */
  double true_residual;   /* max over right-hand sides, FP64 apply             */
  double seconds;
  int64_t applies;        /* Liouvillian applies performed                     */
} heom_solver_report;

/* Defaults: restart 30, max_iter 3000, tol 1e-8, Jacobi, FP64, inner_tol
 * 1e-5, max_refine 20, rhs_chunk 0 (automatic), fallback on. */
void heom_default_opts(heom_solver_opts *o);
/* Frequencies per multi-RHS solve that heom_spectrum uses with options o on
 * hierarchy h (the odd one for a density of states): o->rhs_chunk when
 * positive, else 1 for hierarchies of at least 2^18 elements per column
 * (N d^2) and 16 below.  Size the workspace with n_rhs = this value for a
 * power spectrum and twice it for a density of states.  0 for a NULL h. */
int32_t heom_spectrum_chunk(const heom_hier *h, const heom_solver_opts *o);
/* Device workspace (bytes) that `op` needs with options o (NULL = defaults).
 * n_rhs: for HEOM_OP_SPECTRUM the number of columns of one chunk, i.e.
 * rhs_chunk for a power spectrum and 2 rhs_chunk for a density of states;
 * ignored otherwise. */
heom_status heom_workspace_size(const heom_hier *h, int32_t op, const heom_solver_opts *o, int64_t n_rhs,
                                size_t *bytes);

/* Stationary state of all ADOs (Package architecture, panel (d) of the
 * package figure: M x = 0 for the even-parity HEOMLS of eq:HEOM, normalised
 * by Tr rho_0 = 1).  Solves B x = e_0 where B is M (even parity) with the
 * equation of element (0,0) of ADO 0 replaced by Tr rho_0 = 1.  x_dev:
 * FP64 [N][d][d] (initial guess if o->use_x0).  Synchronises the stream at
 * every convergence check. */
heom_status heom_steady(heom_hier *h, void *x_dev, const heom_solver_opts *o, heom_solver_report *r,
                        void *ws, size_t ws_bytes, void *stream);

/* Spectra (Methods, "Numerical computation of the spectrum").
 * kind 0 = density of states of the fermionic operator `op` (d x d host):
 *   pi A(w) = -Re{Tr[op x_+,0] + Tr[op^dag x_-,0]},
 *   (M_odd + i w) x_+ = op^dag rho_ss, (M_odd - i w) x_- = op rho_ss;
 *   `even` is the even-parity hierarchy of rho_ss, `odd` the odd one.
 * kind 1 = power spectral density of the bosonic operator `op`:
 *   pi S(w) = -Re Tr[op^dag x_0], (M_even - i w) x = op rho_ss; odd = NULL.
 * The right-hand side left-multiplies every ADO of x_ss (FP64, device).
 * out_host: n_omega doubles.  Frequencies are solved rhs_chunk at a time
 * as multi-RHS systems. */
heom_status heom_spectrum(heom_hier *even, heom_hier *odd, const void *x_ss_dev, int32_t kind,
                          const double *op, const double *omega, int64_t n_omega, double *out_host,
                          const heom_solver_opts *o, heom_solver_report *r, void *ws, size_t ws_bytes,
                          void *stream);

/* ------------------------------------------------------------------------
 * Learned block preconditioner
 * ------------------------------------------------------------------------
 * A multilayer perceptron g: features -> 2 d^2 applied to every ADO block
 * of a residual r (not a passage of the paper: the learned part of this
 * library).  With nu_a = |r_a| the features of block a of right-hand side
 * j are [Re r_a / nu_a, Im r_a / nu_a, n_a / n_max, m_a / m_max,
 * Re c_a / cs, Im c_a / cs, Re z_j / cs, Im z_j / cs] (c_a the ADO's decay,
 * z_j the shift of the system, cs = max |c_a|; a zero block has zero block
 * features), padded with zeros to k1 = a multiple of 32, and the
 * preconditioned block is z_a = r_a + nu_a (g_re + i g_im): the untrained
 * (zero) network is the identity, the better plain map of the large
 * fermionic models, and a zero residual block stays zero.  Layers:
 * k1 -> hidden -> hidden -> o_pad (= 2 d^2 rounded up to 32) with ReLU; BF16
 * operands, FP32 accumulation, FP32 master weights.  Parameters are laid
 * out as [W1 (hidden x k1), b1, W2 (hidden x hidden), b2, W3 (o_pad x
 * hidden), b3], row-major FP32.  Networks live on the device current at
 * creation. */

/* Seeded He-uniform initialisation (last layer scaled by 0.05). */
heom_status heom_nn_create(int32_t d, int32_t hidden, uint64_t seed, heom_nn **out);
void heom_nn_free(heom_nn *nn);
heom_status heom_nn_info(const heom_nn *nn, int32_t *k1, int32_t *o_pad, int32_t *n_params);
heom_status heom_nn_get_params(const heom_nn *nn, float *host);
heom_status heom_nn_set_params(heom_nn *nn, const float *host);
heom_status heom_nn_save(const heom_nn *nn, const char *path);
heom_status heom_nn_load(const char *path, heom_nn **out);

/* Training pairs from a residual r (FP64 [N][d][d], device) and the error
 * e = x* - x it leaves (FP64, device, or NULL for features only): writes
 * the BF16 features X [N][k1], the FP32 targets T [N][o_pad] =
 * (e_a - r_a) / nu_a (zero for a zero block and in the padding) and, when
 * W_dev is not NULL, the FP32 row weights W [N] = nu_a^2 / mean_b nu_b^2,
 * so that the weighted loss below measures the error of the correction
 * nu_a g_a against e_a - r_a itself, relative to the pair set's mean.
 * border is kept for the call's form and has no effect. */
heom_status heom_nn_pairs(heom_hier *h, const heom_nn *nn, const void *r_dev, const void *e_dev, int32_t border,
                          void *X_dev, void *T_dev, void *W_dev, void *stream);
/* O [rows][o_pad] FP32 = g(X) for BF16 features X [rows][k1]. */
heom_status heom_nn_forward(const heom_nn *nn, const void *X_dev, int64_t rows, void *O_dev, void *stream);
/* Gradients of sum_rows w (g(X) - T)^2 / (2 rows) in the parameter layout
 * above (host, n_params floats) and the loss (host, 1 float); W_dev: FP32
 * row weights [rows], or NULL for all ones. */
heom_status heom_nn_gradients(const heom_nn *nn, const void *X_dev, const void *T_dev, const void *W_dev, int64_t rows,
                              float *grads_host, float *loss_host, void *stream);
/* Adam (beta 0.9 / 0.999, eps 1e-8) on the weighted loss above over
 * shuffled mini-batches of `batch` rows for `epochs` passes over the
 * training set: all `rows` pairs, or a fixed seeded subset of `subset` of
 * them when 0 < subset < rows.  W_dev may be NULL (all ones).
 * loss_per_epoch (host, epochs floats, may be NULL) receives the mean
 * mini-batch loss.  Allocates its own scratch. */
heom_status heom_nn_train(heom_nn *nn, const void *X_dev, const void *T_dev, const void *W_dev, int64_t rows,
                          int64_t subset, int32_t epochs, int32_t batch, double lr, uint64_t seed,
                          float *loss_per_epoch, void *stream);

/* Vector helpers for building training pairs on the device.
 * heom_steady_residual: r = e_0 - B x (B as in heom_apply_steady_operator;
 * FP64 [N][d][d]).  heom_vector_axpby: y = alpha x + beta y over n complex
 * elements of the given precision (y is not read when beta = 0). */
/* Electronic current from one fermionic lead into the system (Methods,
 * "Electronic current", eq:last), in units e = hbar = 1:
 *   I = i sum_{nu, h, sigma} (-1)^{delta_{nu,-}} Tr[d_sigma^{nu-bar} rho_{|{alpha,nu,h,sigma}}]
 * over the first-level fermionic ADOs (m = 0, n = 1) of x_dev.  The lead is
 * the set of fermionic bath records records[n_rec] (indices into the baths
 * array given to heom_build_hierarchy, e.g. one record per spin of lead
 * alpha).  h: even-parity hierarchy; x_dev: FP64 ADO vector (normally the
 * stationary state of heom_steady).  out: host double[2], the complex
 * current (real for a stationary state; 0 when n_max = 0).  Synchronises
 * the stream; allocates and frees small device buffers for the term list.
 * Errors: HEOM_ERR_ARG for a NULL argument, an odd-parity hierarchy, a bath
 * index out of range, repeated, or of a bosonic bath. */
heom_status heom_current(heom_hier *h, const void *x_dev, int32_t n_rec, const int32_t *records, double *out,
                         void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * current as heom_current, with the term list and the terms' operators kept
 * in a library-owned device array instead of per-call allocations.  No
 * hipMalloc / hipFree; the array (about 1 MB) is held on every GPU the call
 * runs on until the process ends.  Limits: d <= 32 (HEOM_ERR_UNSUPPORTED
 * beyond).  Every call on one GPU shares that array: calls that overlap on
 * one GPU (other threads or streams) race and must be serialised by the
 * caller.  Synchronises the stream; the host arrays it copies from live on
 * the call's stack or in the handle. */
heom_status heom_current_noalloc(heom_hier *h, const void *x_dev, int32_t n_rec, const int32_t *records, double *out,
                                 void *stream);

/* z = P^{-1} r for a fixed preconditioner precond (HEOM_PREC_JACOBI,
 * HEOM_PREC_SCALED or HEOM_PREC_BLOCK), the map the solvers apply on the
 * right.  r_dev, z_dev: device [N][d][d][n_rhs] complex vectors of the given
 * precision, not aliased.  shifts_dev: NULL, or a device array of n_rhs
 * complex doubles (FP64 whatever the precision), the shift z of column r as
 * in heom_apply_shifted.  border = 1 (one right-hand side) preconditions the
 * stationary-state operator of heom_apply_steady_operator (Jacobi divides
 * element (0,0) of ADO 0 by 1; the block map is unchanged).  Asynchronous on
 * stream; the first call on a hierarchy uploads its tables. */
heom_status heom_precondition(heom_hier *h, int32_t precision, int32_t precond, const void *r_dev, void *z_dev,
                              int32_t n_rhs, const void *shifts_dev, int32_t border, void *stream);
heom_status heom_steady_residual(heom_hier *h, const void *x_dev, void *r_dev, void *stream);
heom_status heom_vector_axpby(int32_t precision, const void *x_dev, double alpha, void *y_dev, double beta, int64_t n,
                              void *stream);

/* ------------------------------------------------------------------------
 * Batched instances
 *
 * Many independent hierarchies (each with its own d <= 16, exponents, tiers,
 * Hamiltonian and baths; for example parameter sweeps or ensembles of
 * models) are advanced together: one launch applies eq:HEOM to every
 * instance, and the batched stationary-state solver runs restarted GMRES on
 * all instances at once with per-instance scalars.  The batch vector is the
 * concatenation of the instance vectors ([N_s][d_s][d_s] complex each, in
 * instance order); heom_batch_info returns the element offsets.
 * ---------------------------------------------------------------------- */
typedef struct heom_batch heom_batch;

/* Build a batch over already-built hierarchies (not copied: they must
 * outlive the batch; the batch uploads their device tables on the current
 * device).  Errors: HEOM_ERR_ARG (NULL / n_inst < 1), HEOM_ERR_UNSUPPORTED
 * (an instance with d > 16). */
heom_status heom_batch_create(int32_t n_inst, heom_hier *const *inst, heom_batch **out);
void heom_batch_free(heom_batch *b);
/* offsets: n_inst + 1 element offsets (may be NULL); n_tiles: work tiles of
 * the batched launch; grid, order: the launch configuration in use (grid 0 =
 * one block per tile; order 0 = instance-major tiles, 1 = interleaved,
 * costliest instances first). */
heom_status heom_batch_info(const heom_batch *b, int64_t *offsets, int64_t *n_tiles, int32_t *grid, int32_t *order);
/* The launch shape in use, 8 host ints: tile multiplier of the d <= 4
 * instances, tile multiplier of the d = 8 / 16 instances (a tile holds
 * max(4, 256 / d^2) x that many ADOs), wave formulation for d = 8 (1) or
 * one thread per output element (0), the same for d = 16, persistent grid
 * (0: one workgroup per tile), tile order (0 instance-major, 1
 * interleaved), the H terms of each ADO's own block on the matrix cores for
 * the d = 16 wave instances (1; see HEOM_PLAN_PULL_MFMA) or by sparse
 * gathers (0), and 1 if the last heom_batch_tune took the shape from its
 * cache file. */
heom_status heom_batch_shape(const heom_batch *b, int32_t *shape);
/* Sets the launch shape (the first seven values of heom_batch_shape; the
 * multipliers in {1, 2, 4, 8}, the flags in {0, 1}, grid >= 0; else
 * HEOM_ERR_ARG).  Synchronous (uploads the tile list). */
heom_status heom_batch_set_shape(heom_batch *b, const int32_t *shape);
/* y = M x for every instance in one launch (eq:HEOM; border = 1: the
 * bordered stationary-state operator of each instance, see
 * heom_apply_steady_operator).  x, y: device batch vectors of the given
 * precision, not aliased. */
heom_status heom_batch_apply(heom_batch *b, int32_t precision, const void *x_dev, void *y_dev, int32_t border,
                             void *stream);
/* Autotuner: times heom_batch_apply (reps launches per candidate, after two
 * warm-up launches) over the launch shape of heom_batch_shape -- tile
 * multipliers {1, 2, 4, 8} for small and for wave-sized instances, wave
 * formulation or one thread per element for d = 8 and for d = 16, the
 * persistent grid {one workgroup per tile, 2, 4, 8, 16 per CU}, both tile
 * orders, and sparse or matrix-core H terms for d = 16 -- by two sweeps of
 * coordinate descent from the default shape (1, 1, 1, 1, 0, 0, 0).  Keeps the fastest for all later launches (and
 * for the batch's preconditioners, which walk the same tiles) and reports
 * the default and chosen times (ms per apply).  With the environment
 * variable HEOMX_TUNE_CACHE naming a file, a shape stored there for the
 * same device, precision and instance shapes is used without a search, and
 * a searched shape is appended to it (text, one line per batch shape).
 * Shapes differ in the order of floating-point additions, so results agree
 * to rounding, not bit for bit.  x, y: scratch batch vectors of the
 * precision; y is overwritten.  Synchronises the stream. */
heom_status heom_batch_tune(heom_batch *b, int32_t precision, const void *x_dev, void *y_dev, int32_t reps,
                            double *ms_default, double *ms_best, void *stream);
/* Device workspace bytes for heom_batch_steady with these options. */
heom_status heom_batch_workspace_size(const heom_batch *b, const heom_solver_opts *o, size_t *bytes);
/* Stationary state of every instance (the bordered system of
 * heom_steady, Methods and "Package architecture"): restarted GMRES with a
 * right preconditioner on all instances at once, FP64 or FP32 with FP64
 * iterative refinement (opts.mode), each instance to opts.tol in its true
 * residual.  Instances leave the active set when they converge.  use_graph
 * = 1 captures each Arnoldi step's device work (preconditioner, apply,
 * CGS2, norms, the copy of the coefficients to the host) once per basis size
 * into a hipGraph and replays it.  x_dev: FP64 batch vector (initial guess
 * if opts.use_x0).  r: n_inst reports (status, iterations, refinements,
 * true residual; seconds and applies are batch totals).  Returns
 * HEOM_ERR_NOT_CONVERGED if any instance misses the tolerance.
 * opts.precond: HEOM_PREC_NONE, HEOM_PREC_JACOBI or HEOM_PREC_BLOCK; with
 * opts.fallback = 1 the batched pass stops each instance after at most
 * 20 x opts.restart iterations, and each instance that misses the tolerance
 * is solved again from zero on its own with heom_steady: FP64, block preconditioner, restart
 * 8 x opts.restart (at least 240, at most 1000, fewer when the instance's
 * Krylov basis would exceed 2 GiB), same tol and max_iter; up to eight such
 * solves run at once on host threads, each on a stream of its own.  Its
 * report then carries fell_back = 1 (iterations add up).  The workspace size
 * accounts for that pass; the first such solve on an instance uploads the
 * instance's own device tables. */
heom_status heom_batch_steady(heom_batch *b, void *x_dev, const heom_solver_opts *o, heom_solver_report *r,
                              int32_t use_graph, void *ws, size_t ws_bytes, void *stream);

const char *heom_status_string(heom_status s);
const char *heom_last_error(void);
const char *heom_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HEOM_H */
