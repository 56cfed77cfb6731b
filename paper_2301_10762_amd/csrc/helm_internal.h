// Data structures and constants shared by the HIP kernels and the host engine of
// libhelm (the launchers are declared in helm_launch.h).
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
    Coef cf;
    int np, npan, T;        // padded size, panels per block, steps (nblk * npan)
    int row0, dir, nblk;    // first grid row, +1 (down) or -1 (up), blocks of this front
    int pivot;              // 0: diagonal pivots (flagged if small), 1: partial pivoting in tiles
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
// complex64 blocks keep the same 16 x 16 tiles (256 elements, at the same
// places), with the four values a lane takes in the four MFMA steps of a
// tile next to each other (lane 16 g + r, step q: row 16 I + r, column
// 16 T + 4 q + g), so that two 16-byte loads fetch them
__host__ __device__ inline size_t a_tiled4(int row, int col, int np) {
    return ((size_t)(row >> 4) * (np >> 4) + (col >> 4)) * 256 + (size_t)((col & 3) * 16 + (row & 15)) * 4 +
           ((col >> 2) & 3);
}
// and a block of coupling vectors (np rows x S columns, S padded to 16) as
// 4 x 16 tiles, each the B operand of one step (lane 16 g + r holds row
// 4 K + g, column 16 T + r):
__host__ __device__ inline size_t b_tiled(int row, int col, int np) {
    return ((size_t)(col >> 4) * (np >> 2) + (row >> 2)) * 64 + (row & 3) * 16 + (col & 15);
}
// and for complex64 the same 16 x 16 tiles with a lane's four values of a
// tile adjacent (lane 16 g + r, step q: row 16 K + 4 q + g, column 16 T + r)
__host__ __device__ inline size_t b_tiled4(int row, int col, int np) {
    return ((size_t)(col >> 4) * (np >> 4) + (row >> 4)) * 256 + (size_t)((row & 3) * 16 + (col & 15)) * 4 +
           ((row >> 2) & 3);
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

// The per-front tables of a group: written once per factorisation or solve
// group into a small device buffer by a one-workgroup kernel (they reach it
// as its kernel argument, hence the size limit), then read by every step
// launch of the group, each entry in one round of scalar loads.
struct ChainTab {
    ChainInfo c[MAXB];
};
struct SweepTab {
    SweepInfo c[MAXB];
};
static_assert(sizeof(ChainTab) <= 4000 && sizeof(SweepTab) <= 4000, "tables pass through a kernel argument");

constexpr int RTAP = 16;   // taps per sensor of the restriction tables (4 x 4 bicubic)

}  // namespace helm
