// P2^{-1} = Gamma(alpha, mu)^{-1} (the Hessian preconditioner of the
// section on preconditioning the Hessian, eq (P2)) on the GPU.
//
// Gamma = alpha (Dx^T Dx + Dz^T Dz) + mu I with D_n = (n - 1) bidiag(1, -1)
// (eqs (Gamma), (ThisGamma)).  D_n^T D_n is (n - 1)^2 times the Neumann
// difference Laplacian, whose eigenvectors are the DCT-II basis
// cos(pi p (i + 1/2) / n) with eigenvalues 4 sin^2(pi p / (2 n)).  So with Cx,
// Cz the orthonormal DCT-II matrices, a grid vector Y (nz x nx, x fastest)
// has
//     Gamma^{-1} Y = Cz^T [(Cz Y Cx^T) ./ eig] Cx,
//     eig(q, p) = alpha ((nx-1)^2 4 sin^2(pi p/(2 nx)) + (nz-1)^2 4 sin^2(pi q/(2 nz))) + mu,
// the same operator the paper applies with a sparse Cholesky factor, as four
// dense real products that run on the FP64 matrix cores instead of two
// sequential triangular sweeps.
#include <hip/hip_runtime.h>

#include "helm_device.h"
#include "helm_launch.h"

namespace helm {

// C(r, c) = sum_k A(r, k) B(k, c) [/ div(r, c)] for a batch of products, each
// operand addressed by a row stride, a column stride and a batch stride (0:
// shared by the batch).
struct GemmOp {
    const double* A;
    int64_t sar, sak, sab;
    const double* B;
    int64_t sbk, sbc, sbb;
    double* C;
    int64_t scr, scc, scb;
    const double* div;   // optional, dense M x N with row stride N
    int M, N, K;
};

constexpr int GT = 32;   // output tile 32 x 32 per workgroup, one 16 x 16 quarter per wave
constexpr int GK = 64;   // k-chunk staged in LDS: 16 loads in flight per thread, few serial chunks

__global__ __launch_bounds__(256) void k_gemm_f64(const GemmOp op) {
    __shared__ double sA[GK][GT + 1];   // sA[k][r]
    __shared__ double sB[GK][GT + 1];   // sB[k][c]
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = wv >> 1, wc = wv & 1;
    const int r0 = blockIdx.y * GT, c0 = blockIdx.x * GT;
    const int64_t b = blockIdx.z;
    const double* A = op.A + b * op.sab;
    const double* B = op.B + b * op.sbb;
    const int lr = lane & 15, lg = lane >> 4;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < op.K; k0 += GK) {
        // 32 x 64 elements of each operand, eight per thread, the
        // unit-stride index fastest across the workgroup; all loads of a
        // chunk are issued before the first is stored
        double va[8], vb[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = t + 256 * q;
            int rr, kk;
            if (op.sak == 1) { kk = e & (GK - 1); rr = e >> 6; }
            else { rr = e & (GT - 1); kk = e >> 5; }
            const int gr = r0 + rr, gk = k0 + kk;
            va[q] = (gr < op.M && gk < op.K) ? A[gr * op.sar + gk * op.sak] : 0.0;
            int cc, kb;
            if (op.sbk == 1) { kb = e & (GK - 1); cc = e >> 6; }
            else { cc = e & (GT - 1); kb = e >> 5; }
            const int gc = c0 + cc, gk2 = k0 + kb;
            vb[q] = (gc < op.N && gk2 < op.K) ? B[gk2 * op.sbk + gc * op.sbc] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = t + 256 * q;
            if (op.sak == 1) sA[e & (GK - 1)][e >> 6] = va[q];
            else sA[e >> 5][e & (GT - 1)] = va[q];
            if (op.sbk == 1) sB[e & (GK - 1)][e >> 6] = vb[q];
            else sB[e >> 5][e & (GT - 1)] = vb[q];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4)
            acc = mfma16(sA[kk + lg][16 * wr + lr], sB[kk + lg][16 * wc + lr], acc);
        __syncthreads();
    }
    double* C = op.C + b * op.scb;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = r0 + 16 * wr + acc_row<double>(lg, e);
        const int c = c0 + 16 * wc + lr;
        if (r < op.M && c < op.N) {
            double v = acc[e];
            if (op.div) v /= op.div[(int64_t)r * op.N + c];
            C[r * op.scr + c * op.scc] = v;
        }
    }
}

static void gemm(const GemmOp& op, int batch, hipStream_t st) {
    dim3 grid((op.N + GT - 1) / GT, (op.M + GT - 1) / GT, batch);
    hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, st, op);
}

void launch_gamma_solve(const double* Cx, const double* Cz, const double* eig, int nx, int nz, int nvec,
                        const double* Y, double* X, double* T1, double* T2, hipStream_t st) {
    const int64_t N = (int64_t)nx * nz;
    // T1[j][p] = sum_i Y[j][i] Cx[p][i]
    gemm(GemmOp{Y, nx, 1, N, Cx, 1, nx, 0, T1, nx, 1, N, nullptr, nz, nx, nx}, nvec, st);
    // T2[q][p] = sum_j Cz[q][j] T1[j][p] / eig[q][p]
    gemm(GemmOp{Cz, nz, 1, 0, T1, nx, 1, N, T2, nx, 1, N, eig, nz, nx, nz}, nvec, st);
    // T1[j][p] = sum_q Cz[q][j] T2[q][p]
    gemm(GemmOp{Cz, 1, nz, 0, T2, nx, 1, N, T1, nx, 1, N, nullptr, nz, nx, nz}, nvec, st);
    // X[j][i] = sum_p T1[j][p] Cx[p][i]
    gemm(GemmOp{T1, nx, 1, N, Cx, nx, 1, 0, X, nx, 1, N, nullptr, nz, nx, nx}, nvec, st);
}

}  // namespace helm
