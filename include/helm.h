/*
 * helm.h -- C ABI of the MI355X (gfx950) Helmholtz hot-path library, libhelm.so.
 *
 * The library factors and solves the discrete 2-D Helmholtz systems of
 * Downing, Gazzola, Graham & Spence, "Optimising seismic imaging design
 * parameters via bilevel learning" (arXiv 2301.10762):
 *
 *   A(m, w) = S - w^2 M(m) - i w B(m)                       (App. A.1)
 *
 * on an n_x x n_z node grid (P1 elements with nodal quadrature, i.e. the
 * five-point stencil with halved boundary couplings; M = diag(d_k m_k),
 * B = diag(b_k sqrt(m_k)), first-order impedance boundary condition of
 * eq (forward)).  Each system is factored as a block-tridiagonal LU with one
 * dense n_x x n_x block per grid row, the explicit inverse of every Schur
 * complement being kept so that the sweeps are matrix products.
 *
 * Conventions used by every entry point
 *   - Node k = j*nx + i, x_i = i*hx, z_j = j*hz, j = 0 is the top row.
 *   - Complex vectors are interleaved (re, im) doubles, i.e. complex128.
 *     A block of S vectors is column-major: vector s starts at element s*ld
 *     (ld >= nx*nz, counted in complex elements).
 *   - "_dev" pointers are device (HBM) addresses on the current HIP device;
 *     "_host" pointers are host addresses.  The caller owns all of them.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Work is queued on it; entry points that return a status computed on
 *     the GPU (pivot failures, refinement residuals, phi) synchronise it.
 *   - Return value: HELM_OK (0) or a negative HELM_E* code; a description
 *     of the last error on the calling thread is given by helm_last_error().
 *     No exception crosses the ABI.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, nz;   /* nodes per row, number of rows */
    double hx, hz;    /* grid spacings */
} helm_grid;

/* Opaque factorisation of one A(m, w); owns its device memory. */
typedef struct helm_factor_s* helm_factor_t;

typedef struct {
    int32_t ir_iters;    /* refinement corrections applied (0 for a plain FP64 solve) */
    double max_relres;   /* max over columns of ||b - A x||_2 / ||b||_2 (FP64), or -1 if not measured */
    int32_t bad_block;   /* grid row j of the first failed pivot, -1 if none */
    int32_t bad_row;     /* row inside that block, -1 if none */
    int64_t solves;      /* right-hand sides solved by this call (forward + adjoint) */
} helm_info;

enum { HELM_FP64 = 0, HELM_FP32_IR = 1 };

enum {
    HELM_OK = 0,
    HELM_EINVAL = -1,     /* bad argument: sizes, m_k <= 0 or NaN, node index out of range,
                             source coinciding with a receiver, aliasing B and X */
    HELM_ENOMEM = -2,     /* device allocation failed */
    HELM_ESINGULAR = -3,  /* zero pivot in a diagonal tile of a Schur complement */
    HELM_ENOCONV = -4,    /* refinement did not reach the tolerance in max iterations */
    HELM_EDEVICE = -5     /* HIP runtime error */
};

/* ---- factorisation -------------------------------------------------------
 * helm_factor: factor A(m, w) (App. A.1).  m_dev: nx*nz positive doubles
 * (squared slowness, eq (disc_to_cont) with nodal basis), copied into the
 * factor.  precision: HELM_FP64 (complex128 blocks) or HELM_FP32_IR
 * (complex64 blocks; solves are refined in FP64 to `tol`).  On success *out
 * owns ~nz*np^2*(16 or 8) bytes of HBM, np = nx rounded up to 16.
 * Diagonal tiles use diagonal pivots unless one falls below 1e-2 x max|tile|,
 * in which case the factor is recomputed with partial pivoting inside the
 * tiles.  Returns HELM_ESINGULAR with no factor if a pivot is exactly zero.
 * Synchronises `stream`.                                                   */
int helm_factor(const helm_grid* grid, const double* m_dev, double omega, int precision,
                void* stream, helm_factor_t* out);

/* helm_factor_batch: factor `count` independent systems together (their
 * block chains advance in lockstep inside shared kernel launches).  Grids may
 * differ.  outs[c] receives the factor of (grids[c], m_devs[c], omegas[c]).
 * On failure no factor is returned.  Synchronises `stream`.               */
int helm_factor_batch(int32_t count, const helm_grid* grids, const double* const* m_devs,
                      const double* omegas, int precision, void* stream, helm_factor_t* outs);

/* Bytes of HBM a factor of this grid and precision holds (for admission). */
int helm_factor_bytes(const helm_grid* grid, int precision, size_t* bytes);

/* Releases a factor without waiting for the GPU.  Its device memory goes
 * back to the library's cache in the order of the stream the factor was made
 * on, after the factor's last use by a solve call on any other stream (the
 * solve calls record it; helm_solve_noalloc does not, so work it queued with
 * the factor must be complete before this call).  No call that uses the
 * factor may run concurrently with this one.  NULL is ignored. */
void helm_factor_destroy(helm_factor_t f);

/* ---- solves ----------------------------------------------------------------
 * helm_solve: X = A^{-1} B for S columns (the wavefield of App. A.1,
 * "Computing the wavefield", is the case B = e_s).  helm_adjoint_solve:
 * L = A^{-*} R, the conjugate-transpose solve behind eq (lambda), reusing the
 * same factors.  B/R and X/L: device complex128, column-major with leading
 * dimension ld (>= nx*nz; entries past nx*nz in a column are neither read
 * nor written); X must not overlap B.  S >= 1; S <= 0, ld < nx*nz or
 * overlapping buffers return HELM_EINVAL before any launch.  For an FP32 factor the
 * result is refined in FP64 until max_s ||b_s - A x_s|| / ||b_s|| <= tol
 * (tol <= 0 selects 1e-10), at most 10 corrections, else HELM_ENOCONV.  For
 * an FP64 factor tol > 0 also measures the residual into info (and refines
 * in FP64 if needed).  info may be NULL.  Synchronises when a residual is
 * measured.                                                                 */
int helm_solve(helm_factor_t f, const double* B_dev, double* X_dev, int32_t S, int64_t ld,
               double tol, void* stream, helm_info* info);
int helm_adjoint_solve(helm_factor_t f, const double* R_dev, double* L_dev, int32_t S, int64_t ld,
                       double tol, void* stream, helm_info* info);

/* helm_solve_noalloc: helm_solve for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same arguments, kernels and results as helm_solve
 * (bitwise), but every scratch buffer of the call (sweep coupling vectors,
 * residual partials and norms, the complex64 right-hand side and correction
 * of the refinement, or the complex128 ones of an FP64 refinement) comes
 * from one fixed 256 MiB region of device memory that the library holds on
 * each GPU it runs on until the process ends; the call performs no device
 * allocation or free.  A solve whose scratch would exceed 256 MiB returns
 * HELM_EINVAL before any launch (at 401^2: up to 64 columns with complex64
 * factors; with complex128 factors up to 48 columns when tol > 0, any
 * number otherwise).  The region of the current device is used, so call
 * with the factor's device current.  Every call on one GPU shares that
 * GPU's region: calls that overlap in time on one GPU (other threads, or
 * other streams while an earlier call's kernels still run) race on it.
 * Nothing in the region needs to start at zero.                            */
int helm_solve_noalloc(helm_factor_t f, const double* B_dev, double* X_dev, int32_t S, int64_t ld,
                       double tol, void* stream, helm_info* info);

/* helm_solve_batch: the same as helm_solve for `count` factors at once (the
 * sweeps of all factors share kernel launches).  Bs/Xs/Ss/lds per factor;
 * count >= 1 and every entry valid as for helm_solve, else HELM_EINVAL
 * before any launch.                                                        */
int helm_solve_batch(int32_t count, const helm_factor_t* fs, const double* const* B_devs,
                     double* const* X_devs, const int32_t* S, const int64_t* ld, int adjoint,
                     double tol, void* stream, helm_info* infos);

/* ---- lower-level FWI objective and derivatives ---------------------------
 * helm_misfit_grad: phi and grad phi of eq (phi)/(newphi) by the
 * adjoint-state method (Thm A.1, algorithm "Computing phi, grad phi", App.
 * B.1):  for every frequency w_f and source s,
 *     u = A^{-1} e_s,  eps = d - R u,  lambda = A^{-*} R^* eps,
 *     grad_k += -Re (w^2 d_k + b_k i w / (2 sqrt m_k)) u_k conj(lambda_k),
 *     phi += |eps|^2 / 2,
 * plus 1/2 m^T Gamma m and Gamma m with Gamma = alpha (Dx^T Dx + Dz^T Dz) +
 * mu I (eqs (Gamma), (ThisGamma)).  Receivers and sources are grid nodes
 * (R samples u at the node).  dobs_dev: complex128 [n_omega][S][Nr].
 * omegas_host, src_host, rec_host: host arrays.  grad_dev: nx*nz doubles,
 * overwritten.  *phi_host written on return (synchronises).               */
int helm_misfit_grad(const helm_grid* grid, const double* m_dev, int32_t n_omega,
                     const double* omegas_host, const double* dobs_dev, int32_t S,
                     const int32_t* src_host, int32_t Nr, const int32_t* rec_host,
                     double alpha, double mu, int precision, double tol, void* stream,
                     double* phi_host, double* grad_dev, helm_info* info);

/* helm_gn_hvp: Gauss-Newton products (H^(1) + Gamma) mt_a for n_dir
 * directions (lemma "Adjoint-state formula for multiplication by H^(1)",
 * eqs (defv), (H1v)): per frequency and source
 *     u = A^{-1} e_s,  g~ = (w^2 d + b i w/(2 sqrt m)) u,  v = A^{-1}(g~ mt),
 *     z = A^{-*}(R^* R v),  (H^(1) mt)_j += Re g~_j conj(z_j).
 * mt_dev: doubles [n_dir][nx*nz]; hv_dev: same shape, overwritten.         */
int helm_gn_hvp(const helm_grid* grid, const double* m_dev, int32_t n_omega,
                const double* omegas_host, int32_t S, const int32_t* src_host, int32_t Nr,
                const int32_t* rec_host, int32_t n_dir, const double* mt_dev, double alpha,
                double mu, int precision, double tol, void* stream, double* hv_dev,
                helm_info* info);

/* ---- full Hessian and the Hessian system ---------------------------------
 * A Hessian context holds the lower-level state at one model m: the factors
 * of A(m, w) for every frequency, the wavefields u and, when data are given,
 * the adjoint fields lambda (about 2 * n_omega * S * nx*nz * 16 bytes of HBM
 * besides the factors), so that every product with H costs two batched
 * solves per frequency (the four-solve count of the discussion of the cost
 * of a product with H, u and lambda being shared by all products).
 */
typedef struct helm_hess_s* helm_hess_t;

/* helm_hess_create: factor and solve at m.  With dobs_dev (complex128
 * [n_omega][S][Nr]) the context gives the full Hessian
 *     H = H^(1) + H^(2) + Gamma(alpha, mu)
 * (lemmas "Adjoint-state formula for multiplication by H^(1)" and "... for
 * H^(2)", eqs (H1v), (I6), (Jac_exp)); without data (NULL) it gives the
 * Gauss-Newton H^(1) + Gamma of helm_gn_hvp.  phi_host and grad_dev
 * (optional, data required) receive phi and grad phi as helm_misfit_grad
 * computes them.  Sources may not coincide with receivers when data are
 * given.  info counts the u and lambda solves.  Synchronises `stream`.
 * *out is released with helm_hess_destroy.                                 */
int helm_hess_create(const helm_grid* grid, const double* m_dev, int32_t n_omega,
                     const double* omegas_host, const double* dobs_dev, int32_t S,
                     const int32_t* src_host, int32_t Nr, const int32_t* rec_host, double alpha,
                     double mu, int precision, double tol, void* stream, double* phi_host,
                     double* grad_dev, helm_info* info, helm_hess_t* out);

/* helm_hess_create_at: helm_hess_create with the Nr sensors at points of
 * the domain, rec_xz_host = [Nr][2] doubles (x, z) with 0 <= x <= (nx-1) hx,
 * 0 <= z <= (nz-1) hz, and the sources either at nodes (src_host) or at
 * points (src_xz_host, [S][2], loads as helm_point_sources; exactly one of
 * the two non-NULL); R(P) is the sliding cubic of App. "Numerical
 * restriction operator": (R u)_j is the tensor-product Lagrange cubic through
 * the 4 x 4 nodes nearest to p_j (for p in [x_i, x_{i+1}] the nodes x_{i-1}
 * .. x_{i+2}, moved inward at the edges), so at a node it is the nodal value.
 * Needs nx, nz >= 4.  R^* is its transpose.  Everything else (phi, grad,
 * products, PCG) is as for helm_hess_create.                               */
int helm_hess_create_at(const helm_grid* grid, const double* m_dev, int32_t n_omega,
                        const double* omegas_host, const double* dobs_dev, int32_t S,
                        const int32_t* src_host, const double* src_xz_host, int32_t Nr,
                        const double* rec_xz_host,
                        double alpha, double mu, int precision, double tol, void* stream,
                        double* phi_host, double* grad_dev, helm_info* info, helm_hess_t* out);

/* helm_upper_grad: derivatives of the upper-level objective
 * psi = 1/2 ||m' - m_FWI||^2 (eq (SOobj)) for one training model m', at a
 * context made by helm_hess_create_at at m_FWI with data d = R(P) u(m'):
 *   tau = A(m_FWI)^{-1}(g rho u) (eq (tau_def)), one solve per frequency and source;
 *   dpsi/dp_{j,l} = -sum_{w,s} Re[(d_l tau)(p_j) conj(eps_j)
 *                                + tau(p_j) conj(dd_{j,l} - (d_l u)(p_j))]
 *   (theorem on the derivative with respect to p_{j,l}, eqs (gradALT),
 *   (gradALT1), with the conjugates its derivation gives), eps = d - R u;
 *   dpsi/dalpha = m_FWI^T (Dx^T Dx + Dz^T Dz) rho (eq (sograda)).
 * rho_dev: nx*nz doubles, the solution of H rho = m' - m_FWI (eq (rho),
 * helm_hess_pcg).  ddata_dev: complex128 [n_omega][S][Nr][2], the x and z
 * derivatives of the training wavefield at the sensors, dR/dx_l u(m')
 * (helm_restrict with deriv 1 and 2).  dpsi_dp_host: [Nr][2] doubles
 * (x, z); *dpsi_dalpha_host.  For several training models average the
 * results (the 1/N_m' of eqs (gradALT), (sograda)).  Synchronises
 * `stream`.                                                               */
int helm_upper_grad(helm_hess_t h, const double* rho_dev, const double* ddata_dev, void* stream,
                    double* dpsi_dp_host, double* dpsi_dalpha_host, helm_info* info);

/* helm_point_sources: right-hand sides for S point sources between nodes
 * (App. "Numerical forward model": f = delta_s in the load integral, so
 * f_j = phi_j(s) for the P1 hat functions).  The rectangles' diagonal is
 * not stated, so the loads of the two ways of cutting them are averaged
 * (four nonzeros at the corners of the cell holding s; e_s at a node).
 * src_xz_host: [S][2] points inside the domain.  B_dev: complex128, column s
 * at s*ld, overwritten (zero outside the loads).  Synchronises `stream`.   */
int helm_point_sources(const helm_grid* grid, int32_t S, const double* src_xz_host, double* B_dev,
                       int64_t ld, void* stream);

/* helm_restrict: out = R(P) U (deriv 0) or its derivative with respect to
 * the sensors' x (1) or z (2) coordinate, for S complex128 fields U_dev
 * (column s at s*ld) and Nr sensors at points as for helm_hess_create_at.
 * out_dev: complex128 [S][Nr].  Synchronises `stream`.                    */
int helm_restrict(const helm_grid* grid, int32_t Nr, const double* rec_xz_host, int deriv,
                  const double* U_dev, int32_t S, int64_t ld, double* out_dev, void* stream);

/* helm_hess_apply: hv_a = H mt_a for n_dir directions.  Per frequency and
 * source, with g = w^2 d + b i w / (2 sqrt m) and h = dg/dm = -i w b /
 * (4 m^{3/2}):
 *     v = A^{-1}(g mt u),  z = A^{-*}(R^* R v - conj(g) mt lambda),
 *     hv_j += Re g_j u_j conj(z_j) - Re g_j v_j conj(lambda_j)
 *             - Re h_j mt_j u_j conj(lambda_j),
 * (Gauss-Newton context: z = A^{-*} R^* R v and only the first term), then
 * hv += Gamma mt.  mt_dev, hv_dev: doubles [n_dir][nx*nz], not
 * overlapping; hv overwritten; n_dir * S <= 65535.  Solves use the context's precision and tol.
 * Synchronises `stream`.  Calls on one context must not overlap.           */
int helm_hess_apply(helm_hess_t h, int32_t n_dir, const double* mt_dev, double* hv_dev,
                    void* stream, helm_info* info);

/* helm_hess_pcg: preconditioned conjugate gradients for the Hessian system
 * H x = b (eq (rho)) with the preconditioner P2 = Gamma(p_alpha, p_mu)
 * (eq (P2)); p_mu <= 0 (and p_alpha = 0) runs plain CG.  x_dev holds the
 * start vector on entry (the paper starts from all ones) and the solution on
 * return.  Stops once ||r_n||_2 <= rtol ||r_0||_2 (r_n by the CG recurrence,
 * r_0 = b - H x_0) or after maxit iterations.  P2^{-1} is applied exactly
 * through the eigen-decomposition of Gamma (orthonormal DCT-II in x and z,
 * four FP64 matrix-core products) where the paper uses a Cholesky factor:
 * the same operator.  *iters and *relres report the iterations and the
 * final ||r_n|| / ||r_0||.  Returns HELM_ENOCONV if the tolerance was not
 * reached, or if p.Hp <= 0 (H not positive definite along a direction;
 * x then holds the last iterate).  b_dev, x_dev: nx*nz doubles.           */
int helm_hess_pcg(helm_hess_t h, const double* b_dev, double* x_dev, double p_alpha, double p_mu,
                  double rtol, int32_t maxit, void* stream, int32_t* iters, double* relres,
                  helm_info* info);

/* helm_hess_pcg_batch: helm_hess_pcg for `count` independent Hessian
 * systems H_c x_c = b_c (one per context: for instance one per training
 * model m', each at its own m_FWI), run in lockstep so that the products
 * with all the H_c share their sweep launches.  Each system follows exactly
 * the iteration it would follow alone and leaves the lockstep when it stops.
 * The contexts must share precision and tol, and be distinct.  Per system:
 * iters[c], relres[c] (final ||r_n|| / ||r_0||), status[c] (0 converged,
 * 1 iteration limit, 2 p.Hp <= 0) and infos[c] (each may be NULL).
 * Returns HELM_OK whatever the statuses (they are results).              */
int helm_hess_pcg_batch(int32_t count, const helm_hess_t* hs, const double* const* b_devs,
                        double* const* x_devs, double p_alpha, double p_mu, double rtol,
                        int32_t maxit, void* stream, int32_t* iters, double* relres,
                        int32_t* status, helm_info* infos);

void helm_hess_destroy(helm_hess_t h);

/* helm_gamma_solve: X = Gamma(alpha, mu)^{-1} Y for n grid vectors (eq (P2)
 * with eqs (Gamma), (ThisGamma)), alpha >= 0, mu > 0, by the DCT-II
 * eigen-decomposition described at helm_hess_pcg.  Y_dev, X_dev: doubles
 * [n][nx*nz]; X may equal Y.  Synchronises `stream`.                       */
int helm_gamma_solve(const helm_grid* grid, double alpha, double mu, int32_t n, const double* Y_dev,
                     double* X_dev, void* stream);

/* ---- lower-level FWI ------------------------------------------------------ */

typedef struct {
    int32_t memory;         /* (s, y) pairs kept */
    int32_t max_iters;      /* iterations */
    int32_t max_evals;      /* evaluations per line search */
    double gtol;            /* stop when ||grad|| <= gtol ||grad_0|| */
    double c1, c2;          /* strong Wolfe constants, 0 < c1 < c2 < 1 */
    double first_change;    /* first trial step changes m by first_change * max|m| */
} helm_lbfgs_opts;

typedef struct {
    int32_t iterations, evals;
    int32_t status;         /* 0 converged, 1 iteration limit, 2 line search failed */
    double phi0, phi, gnorm0, gnorm;
    int64_t solves;         /* Helmholtz solves of all evaluations */
} helm_fwi_info;

/* helm_fwi: the lower-level FWI m_FWI = argmin phi(m) (eq (newphi)) by
 * L-BFGS with a strong-Wolfe line search (App. "Optimisation", after
 * Nocedal & Wright): two-loop recursion with initial matrix (s.y/y.y) I;
 * the first step along -grad scaled so that m changes by first_change *
 * max|m|; trial steps 1, 2, 4, .. until the strong Wolfe conditions hold or
 * the minimum is bracketed, then zoom by the cubic interpolation of f, f'
 * at the bracket's ends (bisection when it falls within a tenth of them).
 * A trial model with some m_k <= 0 counts as phi = +inf.  Each evaluation
 * is phi and grad phi as helm_misfit_grad computes them, with source
 * nodes src_host or points src_xz_host and receiver nodes rec_host or
 * sensor points rec_xz_host (exactly one of each pair non-NULL; see
 * helm_hess_create_at).  m_dev: the start model on entry, the result on
 * return (after an error return, the last accepted iterate).  phi_hist_host (optional): max_iters + 1 doubles, phi at every
 * iterate.  The statuses are results, not errors.  Synchronises `stream`. */
int helm_fwi(const helm_grid* grid, double* m_dev, int32_t n_omega, const double* omegas_host,
             const double* dobs_dev, int32_t S, const int32_t* src_host, const double* src_xz_host,
             int32_t Nr, const int32_t* rec_host, const double* rec_xz_host, double alpha, double mu,
             int precision, double tol, const helm_lbfgs_opts* opts, void* stream,
             double* phi_hist_host, helm_fwi_info* info);

/* ---- building blocks exposed for tests and measurement ------------------ */

/* r = B - A(m, w) X (FP64, five-point form of App. A.1) and, per column,
 * ||r||_2^2 and ||B||_2^2 into norms_dev[2*s], norms_dev[2*s+1].  r_dev may
 * be NULL (norms only).  adjoint != 0 uses A^* instead of A.               */
int helm_residual(const helm_grid* grid, const double* m_dev, double omega, int adjoint,
                  const double* B_dev, const double* X_dev, double* r_dev, int32_t S, int64_t ld,
                  double* norms_dev, void* stream);

/* Diagonal-tile Gauss-Jordan inverse of `count` kb x kb complex128 matrices
 * (kb in {16, 32}, row-major, contiguous): the building block of the block
 * factorisation, exposed to test it alone.  pivot = 1: partial pivoting
 * inside the tile; pivot = 0: diagonal pivots, HELM_ESINGULAR if one is
 * below 1e-2 times the largest entry magnitude of the tile.                */
int helm_tile_inverse(int32_t count, int32_t kb, int pivot, const double* A_dev, double* T_dev, void* stream);

/* Diagonal tiles are inverted with diagonal pivots by default; a factor
 * whose tile meets a pivot below 1e-2 x max|tile| is refactored with partial
 * pivoting inside the tiles.  always != 0 selects partial pivoting from the
 * start for every later factorisation (process-wide).                      */
void helm_set_tile_pivoting(int always);

/* Device memory of factors and scratch is recycled through a cache of freed
 * blocks: helm_factor_destroy and the end of every call return their blocks
 * to it (with an event marking their last use on the stream), and a later
 * request of about the same size takes a cached block after queueing a wait
 * on that event.  The cache holds at most `bytes` (default 32 GiB); the
 * oldest blocks beyond the limit go back to the device's memory pool once
 * their last use has finished.  helm_set_cache_limit(0) empties the cache.
 * This memory is outside the helm_factor_bytes() accounting of live factors.
 * Returns the previous limit.  Not for use while another thread is inside
 * the library. */
size_t helm_set_cache_limit(size_t bytes);

/* Lane-layout check of the matrix-core instruction used by the kernels:
 * D = A(16x4) * B(4x16) in FP64 (prec 0) or FP32 (prec 1) on one wavefront. */
int helm_mfma_probe(int prec, const double* A_dev, const double* B_dev, double* D_dev, void* stream);

/* Live timing of the hot kernels with HIP events.  helm_kernel_timing(1)
 * resets the totals and brackets every run of back-to-back launches of one
 * kind (all panel steps of a factorisation group; one forward or backward
 * sweep) with two events on its stream; helm_kernel_time reports, per kind,
 * the summed elapsed milliseconds and the number of launches inside the
 * timed runs (it waits for them), so total / count is the average launch
 * duration.  Kind 0 is the factorisation step (block update + next diagonal
 * tile), kind 1 the initial assembly launch, kind 2 a sweep step.          */
void helm_kernel_timing(int enable);
int helm_kernel_time(int kind, double* total_ms, int64_t* count);

/* Counters since load: 0 = kernel launches, 1 = right-hand-side solves,
 * 4 = bytes of device memory held in the block cache (above); -1 for any
 * other index. */
int64_t helm_counter(int which);

const char* helm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HELM_H */
