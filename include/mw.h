/*
 * mw.h -- C ABI of the MI355X microwave-tomography solve library.
 *
 * Solves, for many antenna right-hand sides at once, the lowest-order
 * Nedelec edge-element discretisation of the time-harmonic Maxwell problem
 *
 *     curl curl E - k0^2 eps_r E = 0 in Omega,   E x n = 0 on metal walls,
 *     (curl E) x n + i beta n x (E x n) = g     on ports / impedance faces
 *
 * (paper: Section 2, problem (pbdirect), variational form (pbdirectvarf),
 * linear systems (linsys) with one matrix A for every antenna), by GMRES
 * right-preconditioned with the one-level Optimized Restricted Additive
 * Schwarz preconditioner  M^-1 = sum_i R_i^T D_i B_i^-1 R_i  (Section 3,
 * equations (algebPartUnity), (chi), (ORAS)), stopped on the unpreconditioned
 * relative residual (Section 6).  It also forms the scattering matrix
 * (Section 4, equation (sij)), the misfit J (equation (defJ)) and its adjoint
 * gradient with respect to a per-tetrahedron permittivity (Section 5,
 * problems (pblin), (pbadj)).
 *
 * Conventions
 *  - time factor e^{+i omega t}: lossy media have Im eps_r < 0;
 *  - complex numbers are two doubles (re, im), layout-compatible with
 *    C99 double _Complex, std::complex<double> and torch.complex128;
 *  - unknowns are the circulations along the oriented mesh edges
 *    (lo -> hi global vertex id), edges numbered in lexicographic (lo, hi)
 *    order; the edges lying on a PEC face are eliminated and the remaining
 *    ("free") edges, in ascending edge order, are the n unknowns;
 *  - multi-vectors (B, X, U, ...) are n x nrhs, row-major, the right-hand-
 *    side index contiguous (an n x nrhs contiguous torch tensor);
 *  - every call returns mw_status; MW_OK is 0, errors are negative; the
 *    message of the last error of the calling thread is mw_last_error().
 *    Nothing throws across the ABI.
 *
 * Ownership: the caller owns every buffer it passes; "host" arrays are read
 * during the call only (copied where kept), "device" pointers must be device
 * memory of the context's device, valid for the duration of the call.  The
 * library owns the factors, Krylov bases and workspaces it allocates; they
 * are released by mw_destroy_problem / mw_destroy.  A problem issues its
 * work on its own stream (the context's stream, mw_set_stream, when it was
 * assembled; mw_problem_set_stream to change it) and every call returns after
 * that stream has finished the call's work.
 */
#ifndef MW_H
#define MW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MW_OK = 0,
  MW_EINVAL = -1,     /* bad argument: NULL, size, index or shape */
  MW_ENOMEM = -2,     /* request exceeds the context's HBM budget; nothing allocated */
  MW_ESINGULAR = -3,  /* zero pivot in a subdomain factorisation (message names it) */
  MW_ENOCONV = -4,    /* GMRES reached maxit; X holds the last iterate, info filled */
  MW_ENUMERIC = -5,   /* NaN or Inf in a GMRES residual (e.g. from the right-hand
                         side) or in a subdomain matrix (from the permittivity) */
  MW_EDEVICE = -6     /* HIP runtime error (message holds its string) */
} mw_status;

typedef enum { MW_C128 = 0, MW_C64 = 1 } mw_precision;
/* Subdomain factorisation: LU with partial pivoting, or L D L^T without
 * interchanges for the complex-symmetric B_i (about half the work); AUTO takes
 * L D L^T when every tetrahedron is lossy (Im eps_r < 0), which makes the
 * imaginary part of every B_i positive definite, so no pivot can vanish. */
typedef enum { MW_FACTOR_AUTO = 0, MW_FACTOR_LU = 1, MW_FACTOR_LDLT = 2 } mw_factorization;
/* Form of the subdomain triangular solves (mw_set_solve_form). */
typedef enum { MW_SOLVE_AUTO = 0, MW_SOLVE_RECURSIVE = 1, MW_SOLVE_ROWS = 2 } mw_solve_form;
/* Precision of the GMRES Krylov basis (mw_set_krylov_basis). */
typedef enum { MW_BASIS_AUTO = 0, MW_BASIS_FP64 = 1, MW_BASIS_FP32_LEAN = 2 } mw_krylov_basis;
/* Coarse space of the two-level preconditioner (mw_set_coarse_space). */
typedef enum { MW_COARSE_NONE = 0, MW_COARSE_CONST = 1 } mw_coarse_space;

#define MW_TAG_PEC (-1)
#define MW_TAG_IMPEDANCE 0
/* btag >= 1 : aperture of port (btag - 1) */

typedef struct { double re, im; } mw_complex;

typedef struct mw_ctx mw_ctx;
typedef struct mw_problem mw_problem;

/* Tetrahedral mesh (host arrays).  Tetrahedra and faces may list their
 * vertices in any order.  bface/btag label every boundary face that carries
 * a condition: PEC (E x n = 0, equation (eqmetal)), impedance with the
 * problem's beta_imp (the chamber top, the first-order absorbing condition
 * of equation (eqwgi)), or a port aperture (equations (eqwgj), (eqwgi)). */
typedef struct {
  int32_t nv;
  const double *xyz;     /* [nv*3] */
  int32_t nt;
  const int32_t *tet;    /* [nt*4] */
  int32_t nbf;
  const int32_t *bface;  /* [nbf*3] */
  const int32_t *btag;   /* [nbf]  */
} mw_mesh;

/* Port k (faces with btag == k+1): propagation constant beta of its
 * fundamental mode and that mode's tangential profile on the aperture,
 *   E0(x) = pol * cos(pi * s / width),  s = radius * wrap(atan2(y,x) - theta),
 * wrap() to (-pi, pi].  Section 2: g = (curl E0) x n + i beta n x (E0 x n),
 * which for the incoming mode is 2 i beta E0_t. */
typedef struct {
  mw_complex beta;
  double radius, theta, width;
  double pol[3];
} mw_port;

typedef struct {
  double tol;        /* stop when ||b - A x||_2 / ||b||_2 <= tol, per column (Section 6) */
  int32_t restart;   /* GMRES restart length m (>= 1) */
  int32_t maxit;     /* max total iterations per column */
  int32_t use_x0;    /* 1: X holds the initial guess on entry; 0: x0 = 0 */
  int32_t block;     /* 0: pseudo-block GMRES (each column its own Krylov space);
                        32: block GMRES, the columns grouped 32 at a time into
                        blocks that share one block Krylov space (Section 7:
                        block methods; Saad, Section 6.12).  Batches take 0. */
} mw_solve_opts;

typedef struct {
  int32_t *iters;    /* host [nrhs] or NULL: iterations per column */
  double *relres;    /* host [nrhs] or NULL: final true relative residual */
  int32_t max_iters; /* out */
  int32_t cycles;    /* out: restart cycles of the slowest chunk */
  int32_t chunks;    /* out: column chunks the solve was split into (memory) */
  double t_solve;    /* out: seconds */
} mw_solve_info;

typedef struct {
  int64_t n;        /* free unknowns */
  int64_t nnz;      /* nonzeros of A */
  int64_t n_edges;  /* all mesh edges */
  int32_t nt, nports;
  int32_t n_sub;    /* 0 until mw_factor_subdomains */
  int64_t sum_ni;   /* sum of local sizes n_i */
  int32_t max_ni;   /* largest n_i */
  int32_t precision;
  int64_t factor_bytes;
  double t_assemble, t_decompose, t_factor; /* seconds of the last calls */
  int32_t factorization; /* of the valid factors: MW_FACTOR_LU or MW_FACTOR_LDLT; 0 if none */
  int64_t state;         /* changes with every call that changes the operator or the factors
                            (mw_update_eps, mw_update_eps_vertex, mw_factor_subdomains,
                            mw_release_factors): solves made at equal states used the same
                            A(eps) and the same factors */
  int32_t coarse_size;   /* unknowns of the coarse problem of the valid factors (0: one-level) */
} mw_problem_info;

/* ---- context -------------------------------------------------------- */
/* device: HIP device ordinal.  hbm_budget_bytes: upper bound on what the
 * library may hold on the device (<= 0: 95 % of the device's memory). */
mw_status mw_create(mw_ctx **out, int device, int64_t hbm_budget_bytes);
/* stream: a hipStream_t of the context's device (NULL = null stream), taken
 * by the problems assembled after this call. */
mw_status mw_set_stream(mw_ctx *ctx, void *stream);
mw_status mw_destroy(mw_ctx *ctx);
const char *mw_last_error(void);

/* ---- assembly (Section 2, (pbdirectvarf); Section 2.1) --------------- */
/* Builds the edge topology, eliminates PEC edges and assembles
 *   A = sum_t (K_t - k0^2 eps_t M_t) + sum_F i beta_F M_F
 * on the device (K_t curl-curl, M_t mass of the Whitney functions, M_F the
 * tangential face mass).  eps_r: host [nt] relative permittivity per
 * tetrahedron.  beta_imp: coefficient of MW_TAG_IMPEDANCE faces. */
mw_status mw_assemble(mw_ctx *ctx, const mw_mesh *mesh, const mw_complex *eps_r, double k0,
                      mw_complex beta_imp, const mw_port *ports, int32_t nports,
                      mw_problem **out);
/* Replaces eps (device [nt] complex) and re-assembles A.  Factors become
 * stale: call mw_factor_subdomains again before mw_solve. */
mw_status mw_update_eps(mw_problem *p, const void *eps_dev);
/* eps_r linear on every tetrahedron (Section 6 discretises kappa = k0^2 eps_r
 * with P1 elements): eps_vertex_dev (device [nv] complex) the values at the
 * mesh vertices; the mass term of tetrahedron t becomes
 * sum_v eps_v int_t l_v N_p . N_q (exact), and the tetrahedron means stand for
 * eps_t wherever a per-tetrahedron value is read (the transmission wavenumber,
 * the choice of factorisation).  Re-assembles A; factors become stale.  A
 * later mw_update_eps returns to one value per tetrahedron. */
mw_status mw_update_eps_vertex(mw_problem *p, const void *eps_vertex_dev);
mw_status mw_problem_get_info(mw_problem *p, mw_problem_info *info);
/* host [n]: edge id of every unknown; host [n_edges*2]: edge end vertices. */
mw_status mw_dof_edges(mw_problem *p, int32_t *edge_of_dof, int32_t *edge_vertices);
/* MW_EINVAL while batches of the problem exist. */
mw_status mw_destroy_problem(mw_problem *p);

/* Copies A in CSR (device buffers: row_ptr int64 [n+1], col int32 [nnz],
 * val complex [nnz]); any pointer may be NULL. */
mw_status mw_get_matrix(mw_problem *p, void *row_ptr, void *col, void *val);

/* ---- right-hand sides ------------------------------------------------ */
/* B (device, n x ntx): column j = 2 i beta_k p_k, k = tx[j] (host), with
 * p_k[e] = int_{Gamma_k} E0_k . N_e by the edge-midpoint rule on each face. */
mw_status mw_rhs_ports(mw_problem *p, int32_t ntx, const int32_t *tx, void *B);
/* B (device, n x np): column j = dir_j . N_e(x_j) (unit point dipole);
 * xyz, dir: host [np*3]; the point lies in the lowest-index tetrahedron
 * whose barycentric coordinates are all >= -1e-12 (MW_EINVAL if none). */
mw_status mw_rhs_dipoles(mw_problem *p, int32_t np, const double *xyz, const double *dir,
                         void *B);

/* ---- preconditioner (Section 3) -------------------------------------- */
/* tet_part: host [nt] subdomain of every tetrahedron, values in [0, n_sub)
 * (the non-overlapping partition T_i; every part non-empty), or NULL for the
 * library's own partition: recursive coordinate bisection of the tetrahedron
 * centroids into parts of floor(nt / n_sub) or one more tetrahedra
 * (mw_host_partition returns it; 1 <= n_sub <= nt).  overlap: delta
 * >= 1 layers of vertex-adjacent tetrahedra.  Builds R_i, the partition of
 * unity D_i (P1 chi_i at edge midpoints), the local matrices B_i with
 * impedance transmission conditions i k (E x n).(v x n) on the interfaces,
 * k = k0 sqrt(Re eps_r) of the owning tetrahedron, and factors every B_i
 * densely in `prec` (MW_C64: complex FP32 factors and triangular solves;
 * MW_C128: complex FP64) by the factorisation mw_set_factorization selects
 * (section 6 of the paper factors the B_i by a symmetric L D L^T). */
mw_status mw_factor_subdomains(mw_problem *p, int32_t n_sub, int32_t overlap,
                               mw_precision prec, const int32_t *tet_part);
/* Two-level preconditioner (the paper's conclusion, Section 7, names a coarse
 * space as the remedy for iteration counts that grow with the number of
 * subdomains, Section 6.1, Table tabscaling).  kind MW_COARSE_CONST: every
 * subdomain i contributes the D_i-weighted edge interpolants of the three
 * constant fields, Z_i = R_i^T D_i Phi_i with Phi_i[l, a] = (x_hi - x_lo)[a]
 * of the edge of local unknown l; E = Z^T A Z (3 n_sub unknowns, at most
 * 8192) is assembled on the device and factored like the B_i, in the same
 * precision and factorisation; the preconditioner becomes
 *     M2^-1 v = M^-1 (v - A q) + q,   q = Z E^-1 Z^T v
 * (deflated form: M2^-1 A is the identity on span Z).  Every solve, batch and
 * mw_apply_preconditioner then uses it; mw_apply_preconditioner_noalloc
 * refuses it (MW_EINVAL).  Takes effect at the next mw_factor_subdomains
 * (the factors are invalid until then).  MW_COARSE_NONE (default): one-level. */
mw_status mw_set_coarse_space(mw_problem *p, int32_t kind);
/* kind: an mw_factorization value, used by the next mw_factor_subdomains
 * (default MW_FACTOR_AUTO).  MW_FACTOR_LDLT on matrices whose pivots can
 * vanish may end in MW_ESINGULAR. */
mw_status mw_set_factorization(mw_problem *p, int32_t kind);
/* How the factors are applied, B_i^-1 = U_i^-1 L_i^-1 (the subdomain solves
 * of equation (ORAS), Section 3).  MW_SOLVE_ROWS: after factoring, every
 * 64-row block keeps its off-diagonal rows multiplied by its inverted
 * diagonal block, and each subdomain's forward and backward sweeps run as
 * one product per block inside one workgroup per (subdomain, column tile),
 * all subdomains in one launch; MW_SOLVE_RECURSIVE: recursive blocked
 * triangular solves whose products spread every subdomain over many
 * workgroups.  MW_SOLVE_AUTO (default): ROWS when n_sub >= 512 (enough
 * independent sweeps to fill the device), else RECURSIVE.  Both give the same
 * operator; results differ by rounding only.  Takes effect at the next
 * mw_factor_subdomains.  MW_EINVAL for an unknown form. */
mw_status mw_set_solve_form(mw_problem *p, int32_t form);
/* Storage of the Arnoldi basis of pseudo-block GMRES (Section 6; mixed
 * precision is not in the paper).  MW_BASIS_AUTO (default): complex FP32
 * when the subdomain factors are FP32, complex FP64 otherwise;
 * MW_BASIS_FP64: always complex FP64.  Every product, dot product, the
 * Hessenberg matrix, the iterate and the true residual stay FP64; an FP32
 * basis only rounds the stored vectors (relative 6e-8), which perturbs the
 * Arnoldi relation of a restart cycle by about that much of the cycle's
 * starting residual, while the stopping test is always taken on the true
 * FP64 residual at the restart.  It halves the bytes of Gram-Schmidt.  With
 * the FP32 basis the operator's inputs M^-1 y_j (y_j the Arnoldi candidates)
 * are rounded to FP32 and kept, so that a restart cycle ends with
 * x += [M^-1 y_0 ...] R^-1 y (R relating the candidates to the basis)
 * instead of one more preconditioner application: the update is consistent
 * with the Arnoldi relation, which saves the iterations the next cycle
 * would spend on the preconditioner's rounding.  MW_BASIS_FP32_LEAN: FP32
 * basis without the kept inputs (m n 8 bytes less per column, one more
 * preconditioner application per cycle), for memory-bound batching.  Block
 * GMRES keeps an FP64 basis.  Takes effect at the next solve.  MW_EINVAL for
 * an unknown kind. */
mw_status mw_set_krylov_basis(mw_problem *p, int32_t kind);
/* Z = M^-1 V for nrhs columns (device n x nrhs). */
mw_status mw_apply_preconditioner(mw_problem *p, int32_t nrhs, const void *V, void *Z);

/* Same result as mw_apply_preconditioner (the same kernels, bit for bit),
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The local
 * vectors live in a fixed buffer of MW_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends; the call makes no
 * allocation of its own (the factors come from mw_factor_subdomains).
 * Requires sum_i n_pad_i * nrhs * (8 for MW_C64, 16 for MW_C128) <=
 * MW_NOALLOC_SCRATCH_BYTES (n_pad_i: n_i rounded up to 64), else MW_EINVAL
 * with the sizes in the message.  Every call on a device shares that
 * device's buffer: calls that overlap in time on one device (other host
 * threads, other streams) race and must be serialised by the caller. */
#define MW_NOALLOC_SCRATCH_BYTES (64ll << 20)
mw_status mw_apply_preconditioner_noalloc(mw_problem *p, int32_t nrhs, const void *V, void *Z);

/* ---- solve ----------------------------------------------------------- */
/* X = A^-1 B for nrhs columns (device n x nrhs each) by ORAS right-
 * preconditioned pseudo-block GMRES(m): each column keeps its own Krylov
 * space, GMRES arithmetic in FP64, true residual recomputed at every
 * restart.  Returns MW_ENOCONV (X = last iterate) if a column misses tol
 * within maxit.  info may be NULL. */
mw_status mw_solve(mw_problem *p, int32_t nrhs, const void *B, void *X, const mw_solve_opts *o,
                   mw_solve_info *info);

/* ---- scattering matrix, misfit and gradient (Sections 4-5) ----------- */
/* S (device nrx x ntx) = conj(p_{rx_i}^T U[:, j]) / nu_{rx_i}; U device n x ntx. */
mw_status mw_s_matrix(mw_problem *p, int32_t nrx, const int32_t *rx, int32_t ntx, const void *U,
                      void *S);
/* nu (host [nports]) = int_{Gamma_k} |E0_k|^2. */
mw_status mw_port_norms(mw_problem *p, double *nu);
/* Reverse mode of eps -> U -> S.  gS (device nrx x ntx): dL/dRe S + i dL/dIm S
 * for a real loss L; U (device n x ntx): forward fields of ports tx.
 * Solves A F = Lambda, Lambda_j = sum_i gS_ij p_{rx_i} / nu_{rx_i}, with the
 * current factors, then grad_eps (device [nt]) = conj(k0^2 sum_j f_j^T M_t u_j),
 * i.e. dL/dRe eps + i dL/dIm eps. */
mw_status mw_adjoint_gradient(mw_problem *p, int32_t ntx, const int32_t *tx, int32_t nrx,
                              const int32_t *rx, const void *U, const void *gS, void *grad_eps,
                              const mw_solve_opts *o, mw_solve_info *info);
/* Forward solve of ports tx, S_sim (device nrx x ntx), J = 1/2 sum |S - S_meas|^2
 * (host double), and grad_eps (device [nt]) by one adjoint solve with the
 * same factors.  S_meas: device nrx x ntx. */
mw_status mw_misfit_gradient(mw_problem *p, int32_t ntx, const int32_t *tx, int32_t nrx,
                             const int32_t *rx, const void *S_meas, double *J, void *S_sim,
                             void *grad_eps, const mw_solve_opts *o);


/* Pieces of mw_adjoint_gradient, for callers that run the adjoint solve
 * themselves (e.g. through a batch):
 *  mw_adjoint_rhs: Lambda (device n x ntx) with column j
 *    sum_i gS_ij p_{rx_i} / nu_{rx_i}  (gS device nrx x ntx; rx host [nrx]);
 *  mw_gradient: grad_eps (device [nt]) = conj(k0^2 sum_j f_j^T M_t u_j) from the
 *    forward fields U and adjoint fields F (device n x ntx each), overwritten;
 *  mw_misfit: gS = S_sim - S_meas and J = 1/2 sum |gS|^2 over count entries
 *    (device arrays; J host), the misfit of Section 4 (equation (defJ)). */
mw_status mw_adjoint_rhs(mw_problem *p, int32_t nrx, const int32_t *rx, int32_t ntx, const void *gS,
                         void *Lambda);
mw_status mw_gradient(mw_problem *p, int32_t ntx, const void *U, const void *F, void *grad_eps);
/* With eps_r given at the vertices: grad_vertex (device [nv]) =
 * dL/dRe eps_v + i dL/dIm eps_v = conj(k0^2 sum_t sum_j f_j^T (int_t l_v N_p . N_q) u_j)
 * from the forward fields U and adjoint fields F (device n x ntx each). */
mw_status mw_gradient_vertex(mw_problem *p, int32_t ntx, const void *U, const void *F, void *grad_vertex);
mw_status mw_misfit(mw_problem *p, int64_t count, const void *S_sim, const void *S_meas, void *gS,
                    double *J);
/* The normalised misfit of Section 5, equation (defJ2): gS = W (S_sim - S_meas)
 * and J = 1/2 sum W |S_sim - S_meas|^2 over count entries, W (device double
 * [count], e.g. 1 / |S_empty|^2) or NULL for weights 1 (= mw_misfit). */
mw_status mw_misfit_weighted(mw_problem *p, int64_t count, const void *S_sim, const void *S_meas, const double *W,
                             void *gS, double *J);

/* ---- outer inversion loop (Section 5) ---------------------------------- */
/* Limited-memory BFGS (Section 5 names L-BFGS; Nocedal and Wright, Numerical
 * Optimization, 2nd ed., Algorithms 7.4 and 7.5): two-loop recursion over the
 * last `mem` pairs (s, y) with s^T y > 1e-12 |s| |y|, H0 = (s^T y / y^T y) I
 * from the latest pair, backtracking line search on the Armijo condition
 * J(x + t d) <= J(x) + c1 t g^T d (t halved, at most max_backtrack tries);
 * the first step is scaled so that it moves the largest entry by step0. */
typedef struct {
  int32_t mem;
  double step0;
  double c1;
  int32_t max_backtrack;
} mw_lbfgs_opts;
/* objective: J(x) and its gradient g (both host, n doubles); MW_OK or an error */
typedef mw_status (*mw_objective_fn)(void *user, const double *x, double *J, double *g);
/* Host routine: `iters` accepted steps from x (host [n], overwritten by the
 * last accepted iterate; fewer steps if a line search fails).  J_hist (host
 * [iters+1]) and x_hist (host [(iters+1) * n]) receive the accepted values
 * (either may be NULL); accepted / evaluations the counts (may be NULL). */
mw_status mw_lbfgs(int64_t n, double *x, int32_t iters, const mw_lbfgs_opts *o, mw_objective_fn f, void *user,
                   double *J_hist, double *x_hist, int32_t *accepted, int32_t *evaluations);

/* The inversion of Section 5 over a relative permittivity e given at the mesh
 * vertices (Section 6 takes kappa = k0^2 eps_r in P1).  One evaluation at e:
 * A(e) with the tetrahedron means of e (p1 = 0) or e integrated exactly in
 * the mass term (p1 = 1, mw_update_eps_vertex); the subdomain factors; the
 * forward solves of the ports tx and S (equation (sij)); the misfit of
 * equation (defJ2), J_d = 1/2 sum_ij |S_ij - S_meas,ij|^2 / |S_empty,ij|^2;
 * one adjoint solve with the weighted residual (problem (pbadj)); the
 * gradient per tetrahedron mapped to the vertices by the transpose of the
 * averaging (p1: the exact vertex form); plus the Tikhonov term
 * (alpha/2) int |grad e|^2, exact for P1 through the P1 stiffness matrix K1
 * (alpha/2 Re(e^H K1 e), gradient alpha K1 e).  The gradient is
 * dJ/dRe e + i dJ/dIm e.  Reuse of the previous evaluation's Krylov
 * solutions across iterations (Section 7 names the recycling of Krylov
 * information): recycle = 1, every column of the forward and adjoint solves
 * starts from its own previous field; recycle = 2, all columns start from the
 * best combination of all previous fields, X0 = U Y with Y minimising
 * ||B - A U Y||_F (its normal equations solved on the host; never a larger
 * starting residual than recycle = 1). */
typedef struct {
  double alpha;
  int32_t p1;
  int32_t recycle;
  int32_t n_sub;
  int32_t overlap;
  int32_t precision;     /* mw_precision of the subdomain factors */
  mw_solve_opts solve;   /* tol, restart, maxit, block of every solve (use_x0 ignored) */
} mw_inversion_opts;
typedef struct {
  int32_t evaluations;
  int64_t solve_columns;  /* forward + adjoint right-hand sides solved */
  double seconds;         /* inside evaluations */
} mw_inversion_info;
typedef struct mw_inversion mw_inversion;
/* mesh: the problem's mesh (host; nv, xyz and tet are read); tet_part: host
 * [nt] partition or NULL (the library's own); S_meas, S_empty: device
 * nrx x ntx complex (copied); tx, rx host port lists.  MW_EINVAL if S_empty
 * has a zero entry. */
mw_status mw_inversion_create(mw_problem *p, const mw_mesh *mesh, const int32_t *tet_part,
                              const mw_inversion_opts *o, int32_t ntx, const int32_t *tx, int32_t nrx,
                              const int32_t *rx, const void *S_meas, const void *S_empty, mw_inversion **out);
/* J (host) and grad (device [nv] complex) at eps_v (device [nv] complex). */
mw_status mw_inversion_objective(mw_inversion *inv, const void *eps_v, double *J, void *grad);
/* mw_lbfgs over x = [Re e; Im e] from eps_v (device [nv], overwritten by the
 * last accepted iterate); J_hist host [iters+1], eps_hist host
 * [(iters+1) x nv] complex (either may be NULL). */
mw_status mw_inversion_run(mw_inversion *inv, const mw_lbfgs_opts *lo, int32_t iters, void *eps_v, double *J_hist,
                           void *eps_hist, int32_t *accepted, int32_t *evaluations);
/* Mean GMRES iterations of the forward and adjoint solves of the first cap
 * evaluations (host [cap] each, either may be NULL), and the totals. */
mw_status mw_inversion_get_info(mw_inversion *inv, int32_t cap, double *iters_forward, double *iters_adjoint,
                                mw_inversion_info *info);
mw_status mw_inversion_destroy(mw_inversion *inv);

/* ---- serving: memory, streams, factor cache, continuous batching ------ */
/* Budget and bytes currently held by the context (either pointer may be NULL). */
mw_status mw_ctx_get_info(mw_ctx *ctx, int64_t *budget, int64_t *used);
/* Issue this problem's work on `stream` (a hipStream_t of the context's
 * device) from now on; waits for the problem's previous stream first.
 * Different problems may be driven concurrently from different host threads,
 * each on its own stream; calls on one problem (and its batches) must not
 * overlap. */
mw_status mw_problem_set_stream(mw_problem *p, void *stream);
/* Frees the subdomain factors and solve workspaces (the decomposition is
 * kept, so mw_factor_subdomains with the same partition only refills and
 * refactors).  Batches stay valid but cannot cycle until the factors are
 * rebuilt. */
mw_status mw_release_factors(mw_problem *p);
/* Bytes mw_factor_subdomains holds for the factors of this partition in
 * `prec` (the decomposition must have been built once): banded storage when
 * the next factorisation is L D L^T without interchanges (mw_set_factorization,
 * or automatic with every tetrahedron lossy), dense n_pad^2 per subdomain for
 * LU with interchanges. */
mw_status mw_factor_bytes(mw_problem *p, int32_t n_sub, int32_t overlap, mw_precision prec,
                          const int32_t *tet_part, int64_t *bytes);

/* A batch runs the pseudo-block GMRES(m) of mw_solve over a changing set of
 * columns: requests join between restart cycles and leave at the restart
 * where all their columns have met the tolerance (or maxit).  Every column
 * follows exactly the iteration it would follow alone: x0 = 0, restart m,
 * true FP64 residual at each restart (Section 6).  The batch holds B and X of
 * max_cols column slots (device, 2 x 16 n bytes per slot) and, while columns
 * are active, the Krylov workspaces of the active width (mw_batch_info
 * bytes_per_col each; released when the batch idles). */
typedef struct mw_batch mw_batch;
typedef struct {
  int32_t max_cols, free_cols, active_cols;
  int32_t requests;     /* joined and not yet taken */
  int32_t finished;     /* finished, waiting for mw_batch_take */
  int64_t cycles;       /* restart cycles run so far */
  int64_t slot_bytes;   /* device bytes of the column slots */
  int64_t work_bytes;   /* device bytes of the workspaces held now */
  int64_t bytes_per_col;/* workspace bytes per active column */
} mw_batch_info;
/* o: tol, restart, maxit (use_x0 must be 0); NULL = defaults of mw_solve. */
mw_status mw_batch_create(mw_problem *p, int32_t max_cols, const mw_solve_opts *o, mw_batch **out);
/* Copies B (device n x ncols) into free slots under `tag` (>= 0, unique among
 * the batch's requests); the columns start at the next mw_batch_cycle.
 * MW_ENOMEM if fewer than ncols slots are free (nothing changes). */
mw_status mw_batch_join(mw_batch *b, int64_t tag, int32_t ncols, const void *B);
/* One restart cycle (at most m Arnoldi steps) of every active column, then
 * the true residual of each; requests whose columns have all stopped become
 * finished.  n_active: columns that ran; n_finished: requests finished by
 * this cycle (either may be NULL). */
mw_status mw_batch_cycle(mw_batch *b, int32_t *n_active, int32_t *n_finished);
/* Oldest finished request not yet taken: *tag = -1 if none. */
mw_status mw_batch_poll(mw_batch *b, int64_t *tag, int32_t *ncols);
/* Copies a finished request's solution into X (device n x ncols) and frees
 * its slots; iters, relres: host [ncols] or NULL.  MW_ENOCONV / MW_ENUMERIC
 * (X still written) if a column missed the tolerance or hit NaN/Inf. */
mw_status mw_batch_take(mw_batch *b, int64_t tag, void *X, int32_t *iters, double *relres);
mw_status mw_batch_get_info(mw_batch *b, mw_batch_info *info);
mw_status mw_batch_destroy(mw_batch *b);

/* ---- host-only inspection (no device needed) ------------------------- */
/* Topology the library builds for `mesh` (Section 2.1): number of unknowns,
 * nonzeros of A's pattern, edges; optional host outputs (pass NULL to skip):
 * edge_of_dof [n], row_ptr [n+1], col [nnz]. */
mw_status mw_host_topology(const mw_mesh *mesh, int64_t *n, int64_t *nnz, int64_t *n_edges,
                           int32_t *edge_of_dof, int64_t *row_ptr, int32_t *col);
/* Overlapping decomposition (Section 3) for tet_part: n_loc [n_sub] local
 * sizes, n_faces [n_sub] faces carrying a boundary or transmission term
 * (NULL to skip), and concatenated over subdomains (NULL to skip): sub_dof
 * [sum n_loc] global unknown of each local one (R_i), D [sum n_loc] the
 * partition-of-unity weights.  Within a subdomain the unknowns are in the
 * order of the local matrix and its factors: reverse Cuthill-McKee on the
 * graph of B_i (two unknowns coupled when they share a tetrahedron). */
mw_status mw_host_decomposition(const mw_mesh *mesh, const int32_t *tet_part, int32_t n_sub,
                                int32_t overlap, int32_t *n_loc, int64_t *n_faces, int32_t *sub_dof,
                                double *D);
/* Block least squares of block GMRES (blocks of 32 columns; Saad, Iterative
 * Methods for Sparse Linear Systems, Section 6.12), as the solver runs it on
 * the host: S0 (32 x 32, upper triangular) the starting block's factor,
 * width <= 32 the block's real columns (later ones are padding); H
 * ((steps+1)*32 x steps*32, row-major, leading dimension steps*32) a block
 * upper Hessenberg matrix whose sub-diagonal blocks are upper triangular.
 * Adds the block columns one at a time; resid [steps x 32] (NULL to skip)
 * gets the least-squares residual norm of every right-hand side after each
 * step, Y [steps*32 x 32] (NULL to skip) the final solution of
 * min ||E_1 S0 - H Y||.  Also, for G (32 x 32 Hermitian) given in place of
 * H with steps = 0: resid[0] gets the number of pivots of its Cholesky
 * factor that are <= thr (relative to the largest diagonal entry) and Y its
 * Cholesky factor R (G = R^H R, upper triangular). */
/* Storage of the subdomain factors for this decomposition, in complex
 * elements over all subdomains: dense_elems = sum n_pad^2 (LU with
 * interchanges), band_elems (L D L^T without interchanges: every 64-row
 * block keeps the columns of its structural envelope, 64-aligned, and at
 * least 64 columns past its diagonal block).  blk_lo / blk_hi (host
 * [n_pad(sub)/64], either may be NULL): the stored column range
 * [lo, hi) of every 64-row block of subdomain `sub`. */
mw_status mw_host_factor_storage(const mw_mesh *mesh, const int32_t *tet_part, int32_t n_sub, int32_t overlap,
                                 int32_t sub, int32_t *blk_lo, int32_t *blk_hi, int64_t *dense_elems,
                                 int64_t *band_elems);
/* The partition mw_factor_subdomains takes when tet_part is NULL: tet_part
 * (host [nt], caller-owned) gets the part of every tetrahedron.  Section 3
 * starts from a non-overlapping partition of the mesh into n_sub subdomains;
 * here it is recursive coordinate bisection of the centroids: split across
 * the axis of largest extent, the lower floor(count * floor(np/2) / np) by
 * (coordinate, tetrahedron id) to the first half of the np parts.  MW_EINVAL
 * unless 1 <= n_sub <= nt. */
mw_status mw_host_partition(const mw_mesh *mesh, int32_t n_sub, int32_t *tet_part);
mw_status mw_host_block_lstsq(int32_t steps, int32_t width, const mw_complex *S0, const mw_complex *H,
                              double thr, double *resid, mw_complex *Y);
const char *mw_host_last_error(void);

/* ---- kernel timing (measurement) --------------------------------------- */
/* When enabled, HIP events are recorded on the launch stream around every
 * launch of each kernel family, with the algorithmic flops and HBM bytes of
 * the launch (from the true, unpadded subdomain sizes).  Families are
 * numbered 0 .. mw_timer_families()-1, named by mw_timer_name(). */
int32_t mw_timer_families(void);
const char *mw_timer_name(int32_t family);
void mw_timer_enable(int32_t on);
void mw_timer_reset(void);
/* launches, total milliseconds, flops and bytes since the last reset. */
mw_status mw_timer_read(int32_t family, int64_t *launches, double *ms, double *flops, double *bytes);

#ifdef __cplusplus
}
#endif
#endif /* MW_H */
