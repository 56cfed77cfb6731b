// Host-side launchers of the kernels of libhelm, one per kernel family,
// called by the host engine (helm_host.hip).
#pragma once
#include "helm_internal.h"

namespace helm {

// workgroups per chain of the factorisation launches
int factor_init_blocks(int np);
int factor_step_blocks(int np);
// The per-front tables are read by the kernels from device memory: the host
// writes a group's table once (launch_put_*_table, a one-workgroup copy in
// stream order) and every launch of the group reads it there.
void launch_put_chain_table(const ChainTab& tab, ChainTab* dst, hipStream_t st);
void launch_put_sweep_table(const SweepTab& tab, SweepTab* dst, hipStream_t st);
void launch_factor_init(const ChainTab* dtab, int n, int total_blocks, bool fp32, hipStream_t st);
// uni: factor_uniform() of the group's table (every front has uni workgroups, or 0)
int factor_uniform(const ChainTab& tab, int n);
void launch_factor_step(const ChainTab* dtab, int n, int t, int uni, int total_blocks, bool fp32, hipStream_t st);
// y = b_{row0} (conjugated for adjoint solves) into Y0 of every front
void launch_sweep_init(const SweepTab* dtab, int n, int total_blocks, bool fp32, bool conj_b, hipStream_t st);
// forward step t: row row0 + dir * t of each front; backward step t: row
// brow0 - dir * t.  `groups` row tiles (16 rows) over all fronts, `st` column
// tiles (16 columns).
// uni: sweep_uniform() of the group's table (every front has uni row tiles, or 0)
int sweep_uniform(const SweepTab& tab, int n);
// unroll: sweep_unroll() of the largest padded block size np of the group
int sweep_unroll(int np_max);
void launch_sweep(const SweepTab* dtab, int n, int t, int uni, int unroll, int groups, int st, bool fp32,
                  bool forward, bool conj_b, hipStream_t st_);
int sweep_row_tiles(int np);
int sweep_col_tiles(int S);
void launch_check_model(const double* m, int64_t n, int* flag, hipStream_t st);
void launch_residual(const Coef& cf, int adjoint, const double* B, int64_t ldb, const double* X,
                     int64_t ldx, double* R, int64_t ldr, float* R32, int S, double* partial,
                     int nblk, hipStream_t st);
void launch_norms_finish(const double* partial, int nblk, int S, double* norms, hipStream_t st);
void launch_c128_to_c64(const double* src, int64_t lds, float* dst, int64_t ldd, int64_t N, int S,
                        int conj, hipStream_t st);
void launch_c64_to_c128(const float* src, int64_t lds, double* dst, int64_t ldd, int64_t N, int S,
                        int conj, int accumulate, hipStream_t st);
void launch_conj_inplace(double* X, int64_t ld, int64_t N, int S, hipStream_t st);
void launch_axpy_c128(const double* D, int64_t ldd, double* X, int64_t ldx, int64_t N, int S,
                      hipStream_t st);
void launch_unit_sources(double* E, int64_t ld, int64_t N, const int* nodes, int S, hipStream_t st);
void launch_grad(const Coef& cf, const double* U, int64_t ldu, const double* L, int64_t ldl, int S,
                 double* g, hipStream_t st);
void launch_gn_rhs(const Coef& cf, const double* U, int64_t ldu, int S, const double* mt, int n_dir,
                   double* V, int64_t ldv, hipStream_t st);
void launch_hv(const Coef& cf, const double* U, int64_t ldu, int S, const double* Z, int64_t ldz,
               int n_dir, double* hv, int64_t N, hipStream_t st);
void launch_misfit(const double* U, int64_t ldu, const double* dobs, const int* node, const double* w, int ntap,
                   int Nr, int S, double* eps, double* phi_part, hipStream_t st);
void launch_point_sources(double* E, int64_t ld, const double* xz, int S, int nx, int nz, double hx, double hz,
                          hipStream_t st);   // columns zeroed beforehand
void launch_restrict(const double* U, int64_t ldu, const int* node, const double* w, int ntap, int Nr, int cols,
                     double* out, int64_t ldo, hipStream_t st);
void launch_restrict_adj(const double* Z, int64_t ldz, const int* tnode, const int* tptr, const int* tq,
                         const double* tw, int nt, int cols, double* out, int64_t ldo, hipStream_t st);
void launch_upper(const double* Tau, const double* U, int64_t ld, int S, const double* eps, const double* dd,
                  const int* node, const double* w0, const double* wx, const double* wz, int Nr, double* dp,
                  hipStream_t st);
void launch_zeta_rhs(const Coef& cf, const double* L, int64_t ldl, int S, const double* mt, int n_dir, double* W,
                     int64_t ldw, hipStream_t st);
void launch_hv_full(const Coef& cf, const double* U, const double* L, int64_t ldu, int S, const double* V,
                    const double* Z, int64_t ldz, const double* mt, int n_dir, double* hv, hipStream_t st);
int dot_blocks(int64_t n);
void launch_dot(const double* x, const double* y, int64_t n, double* part, double* out, hipStream_t st);
void launch_absmax(const double* x, int64_t n, double* part, hipStream_t st);   // dot_blocks(n) partial maxima
void launch_lincomb(double* out, double a, const double* x, double b, const double* y, int64_t n, hipStream_t st);
// Gamma(alpha, mu)^{-1} on nvec grid vectors by its eigen-decomposition:
// Cx (nx x nx) and Cz (nz x nz) orthonormal DCT-II matrices, eig (nz x nx)
// the eigenvalues; T1, T2 are nvec * nx * nz scratch; X may equal Y.
void launch_gamma_solve(const double* Cx, const double* Cz, const double* eig, int nx, int nz, int nvec,
                        const double* Y, double* X, double* T1, double* T2, hipStream_t st);
void launch_gamma(const double* m, int nx, int nz, double alpha, double mu, double* g, double* part,
                  int nblk, hipStream_t st);
void launch_sum_scalar(const double* part, int n, double* out, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);
void launch_tile_inverse(int count, int kb, int pivot, const double* A, double* T, int* status, hipStream_t st);
void launch_mfma_probe(int prec, const double* A, const double* B, double* D, hipStream_t st);

}  // namespace helm
