// Internal declarations shared by the HIP kernels and the host engine of libhelm.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace helm {

constexpr int MAXB = 16;   // chains (independent systems) per batched launch
constexpr int TILE = 64;   // output tile of the rank-kb update (64 x 64)
constexpr int KB = 32;     // panel width (columns eliminated per Gauss-Jordan step)

// Everything needed to assemble A(m, w) on the fly (App. A.1).
struct Coef {
    const double* m;   // squared slowness, nx*nz, device
    double omega, hx, hz;
    int nx, nz;
};

// One chain (one system) of a batched factorisation.  The table lives in
// device memory; the launch for global step t makes every chain with t < T
// do panel p = t % npan of block j = t / npan.
struct ChainInfo {
    void* G;        // nz blocks of np x np row-major complex; block j ends as D_j^{-1}
    void* P0;       // ping-pong working blocks (np x np) between panel steps
    void* P1;
    void* Tb;       // two KB x KB slots holding the inverted diagonal tile,
                    // transposed (Tt[c][k] = T[k][c]); step t reads slot t&1
    int* status;    // [0] zero-pivot flag, [1] block, [2] row, [3] small-pivot flag
    Coef cf;
    int np, npan, T;        // padded size, panels per block, steps (nz * npan)
    int pivot;              // 0: diagonal pivots (flagged if small), 1: partial pivoting in tiles
    int utile0;             // first workgroup of this chain in a step launch
    int itile0;             // first workgroup in the initial launch
};

// One chain of a batched block sweep.  The coupling vectors y_j = b_j -
// E w_{j-1} (forward) and z_j = E x_{j+1} (backward) are produced by the
// workgroups that compute the rows they depend on and kept in two ping-pong
// buffers of np x S (column-major, leading dimension np, zero below nx).
struct SweepInfo {
    const void* G;  // factor blocks
    const void* B;  // right-hand sides, column-major (ldb)
    void* X;        // solution being built, column-major (ldx)
    void* Y0;       // coupling vectors, ping-pong
    void* Y1;
    int64_t ldb, ldx;
    int S, nx, nz, np;
    double cz;      // hx / hz: the z-edge coupling is -cz (halved at i = 0, nx-1)
    int tile0, tiles_s;     // first row tile (of 16 rows) of this chain, its column tiles
    int itile0;             // first workgroup of the initial launch
};

// workgroups per chain of the factorisation launches
int factor_init_blocks(int np);
int factor_step_blocks(int np);
void launch_factor_init(const ChainInfo* tab, int n, int total_blocks, bool fp32, hipStream_t st);
void launch_factor_step(const ChainInfo* tab, int n, int t, int total_blocks, bool fp32, hipStream_t st);
// y_0 = b_0 (conjugated for adjoint solves) into Y0 of every chain
void launch_sweep_init(const SweepInfo* tab, int n, int total_blocks, bool fp32, bool conj_b, hipStream_t st);
// forward: step t is block j = t; backward: step t is block j = nz - 2 - t.
// `groups` row tiles (16 rows) over all chains, `st` column tiles (16 columns).
void launch_sweep(const SweepInfo* tab, int n, int t, int groups, int st, bool fp32, bool forward,
                  bool conj_b, hipStream_t st_);
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
void launch_misfit(const double* U, int64_t ldu, const double* dobs, const int* rec, int Nr, int S,
                   double* eps, double* phi_part, hipStream_t st);
void launch_scatter_adj(const double* eps, const int* rec, int Nr, int S, double* R, int64_t ldr,
                        hipStream_t st);
void launch_grad(const Coef& cf, const double* U, int64_t ldu, const double* L, int64_t ldl, int S,
                 double* g, hipStream_t st);
void launch_gn_rhs(const Coef& cf, const double* U, int64_t ldu, int S, const double* mt, int n_dir,
                   double* V, int64_t ldv, hipStream_t st);
void launch_sample_scatter(const double* V, int64_t ldv, const int* rec, int Nr, int cols, double* RV,
                           int64_t ldr, hipStream_t st);
void launch_hv(const Coef& cf, const double* U, int64_t ldu, int S, const double* Z, int64_t ldz,
               int n_dir, double* hv, int64_t N, hipStream_t st);
void launch_gamma(const double* m, int nx, int nz, double alpha, double mu, double* g, double* part,
                  int nblk, hipStream_t st);
void launch_sum_scalar(const double* part, int n, double* out, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);
void launch_tile_inverse(int count, int kb, int pivot, const double* A, double* T, int* status, hipStream_t st);
void launch_mfma_probe(int prec, const double* A, const double* B, double* D, hipStream_t st);

}  // namespace helm
