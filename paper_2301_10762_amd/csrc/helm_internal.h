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

// One front of a batched factorisation.  A system is factored from both
// ends ("twisted"): a top front runs down rows 0, 1, .., k and a bottom front
// up rows nz-1, nz-2, .., k+1, each forming D_next = A_next - E G E.  The
// bottom front finishes earlier and leaves A_k - E G_{k+1} E in a merge
// block, which the top front uses in place of A_k when it forms D_k, so
// G_k is the inverse of the full Schur complement at row k.  The launch for
// global step t makes every front with
// t < T do panel p = t % npan of its block jl = t / npan (grid row
// row0 + dir * jl).
struct ChainInfo {
    void* G;        // nz blocks of np x np complex: D_j row-major while block j is
                    // factored, then its inverse G_j in the A-operand layout (a_tiled)
    void* P0;       // ping-pong working blocks (np x np) between panel steps
    void* P1;
    void* Tb;       // two KB x KB slots holding the inverted diagonal tile,
                    // transposed (Tt[c][k] = T[k][c]); step t reads slot t&1
    int* status;    // [0] zero-pivot flag, [1] block, [2] row, [3] small-pivot flag
    void* Aout;     // bottom front: receives A_next - E G E after its last block
    const void* Ain;   // top front: replaces A of its last block (the merge block)
    // persistent path: the exchange between the front's workgroups
    void* PC;       // panel columns, 2 x (np x 32)
    void* PR;       // panel rows, 2 x (32 x np)
    void* DB;       // next diagonal blocks, 2 x (32 x 32)
    int* ctr;       // rounds completed by the front's workgroups
    const int* peer;   // top front: the bottom front's counter (merge block ready at peer_target)
    int peer_target;
    Coef cf;
    int np, npan, T;        // padded size, panels per block, steps (nblk * npan)
    int row0, dir, nblk;    // first grid row, +1 (down) or -1 (up), blocks of this front
    int pivot;              // 0: diagonal pivots (flagged if small), 1: partial pivoting in tiles
    int utile0;             // first workgroup of this front in a persistent launch
    int ftile0;             // first update workgroup of this front in a step launch, counted
                            // after the one next-tile workgroup per front that leads the grid
    int itile0;             // first workgroup in the initial launch
};

// Matrix-core operand layouts of the sweep data.  A factor block G_j (np x np)
// is stored as 16 x 4 tiles, each the A operand of one 16x16x4 MFMA step in
// lane order (lane l = 16 g + r holds row 16 I + r, column 4 K + g):
__host__ __device__ inline size_t a_tiled(int row, int col, int np) {
    return ((size_t)(row >> 4) * (np >> 2) + (col >> 2)) * 64 + (col & 3) * 16 + (row & 15);
}
// and a block of coupling vectors (np rows x S columns, S padded to 16) as
// 4 x 16 tiles, each the B operand of one step (lane 16 g + r holds row
// 4 K + g, column 16 T + r):
__host__ __device__ inline size_t b_tiled(int row, int col, int np) {
    return ((size_t)(col >> 4) * (np >> 2) + (row >> 2)) * 64 + (row & 3) * 16 + (col & 15);
}

// Row k at which the two fronts of an nz-row system meet (the top front ends
// there), or nz - 1 when there is no bottom front.  The bottom front has
// nz - 1 - k < k blocks, so it ends at least one launch before the top front
// needs its merge block.
__host__ __device__ inline int twist_row(int nz) {
    const int k = (nz + 1) / 2;
    return (nz - 1 - k >= 1) ? k : nz - 1;
}

// One front of a batched block sweep.  Forward: w_j = G_j y_j and the next
// coupling vector y_{j+dir} = b_{j+dir} - E w_j; backward: x_j = w_j - G_j z_j
// and z_{j-dir} = E x_j.  Coupling vectors are produced by the workgroups
// that compute the rows they depend on and kept in two ping-pong buffers of
// np x S16 in the B-operand layout (b_tiled; zero below nx).  With a bottom
// front, its last forward step leaves b_k - E w_{k+1} in `Mout`, which the
// top front reads in place of b_k; the top front's last forward step gives
// x_k and starts both backward sweeps with E x_k (its own buffer and `Zp`).
struct SweepInfo {
    const void* G;  // factor blocks
    const void* B;  // right-hand sides, column-major (ldb)
    void* X;        // solution being built, column-major (ldx)
    void* Y0;       // coupling vectors, ping-pong
    void* Y1;
    const void* Bm; // top front: b_k replaced by the bottom front's b_k - E w_{k+1}
    void* Mout;     // bottom front: where that vector goes
    void* Zp;       // top front: the bottom front's first backward input
    int64_t ldb, ldx;
    int S, nx, nz, np;
    double cz;      // hx / hz: the z-edge coupling is -cz (halved at i = 0, nx-1)
    int row0, dir, nfwd;    // forward: rows row0 + dir * t, t < nfwd
    int brow0, nbwd;        // backward: rows brow0 - dir * t, t < nbwd
    int tile0, tiles_s;     // first row tile (of 16 rows) of this front, its column tiles
    int itile0;             // first workgroup of the initial launch
};

// The per-front tables travel as kernel arguments (by value), so a
// workgroup finds its front and reads its fields without a dependent load
// through a device pointer.
struct ChainTab {
    ChainInfo c[MAXB];
};
struct SweepTab {
    SweepInfo c[MAXB];
};
static_assert(sizeof(ChainTab) <= 4000 && sizeof(SweepTab) <= 4000, "kernel argument tables too large");

// workgroups per chain of the factorisation launches
int factor_init_blocks(int np);
int factor_step_blocks(int np);
void launch_factor_init(const ChainTab& tab, int n, int total_blocks, bool fp32, hipStream_t st);
void launch_factor_step(const ChainTab& tab, int n, int t, int total_blocks, bool fp32, hipStream_t st);
// the whole factorisation in one launch (every workgroup resident; see
// factor_persist_capacity); *err is set if a workgroup's wait timed out
void launch_factor_persist(const ChainTab& tab, int n, int total_blocks, bool fp32, int* err, hipStream_t st);
int factor_persist_capacity(bool fp32);   // resident workgroups of the persistent kernel, 0 if unknown
// y = b_{row0} (conjugated for adjoint solves) into Y0 of every front
void launch_sweep_init(const SweepTab& tab, int n, int total_blocks, bool fp32, bool conj_b, hipStream_t st);
// forward step t: row row0 + dir * t of each front; backward step t: row
// brow0 - dir * t.  `groups` row tiles (16 rows) over all fronts, `st` column
// tiles (16 columns).
void launch_sweep(const SweepTab& tab, int n, int t, int groups, int st, bool fp32, bool forward,
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
void launch_grad(const Coef& cf, const double* U, int64_t ldu, const double* L, int64_t ldl, int S,
                 double* g, hipStream_t st);
void launch_gn_rhs(const Coef& cf, const double* U, int64_t ldu, int S, const double* mt, int n_dir,
                   double* V, int64_t ldv, hipStream_t st);
void launch_hv(const Coef& cf, const double* U, int64_t ldu, int S, const double* Z, int64_t ldz,
               int n_dir, double* hv, int64_t N, hipStream_t st);
constexpr int RTAP = 16;   // taps per sensor of the restriction tables (4 x 4 bicubic)
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
