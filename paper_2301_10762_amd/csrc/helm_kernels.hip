// HIP kernels of libhelm for gfx950 (CDNA4).
//
// The discrete operator (App. A.1 of arXiv 2301.10762) is
//     A(m, w) = S - w^2 diag(d m) - i w diag(b sqrt m),
// with S the five-point stiffness (x-edge coupling hz/hx, z-edge coupling
// hx/hz, halved on boundary edges), d the nodal mass weights (hx*hz, halved
// per boundary direction) and b the boundary-edge weights.  Grouping the
// unknowns by grid row j makes A block tridiagonal: diagonal blocks A_j are
// tridiagonal n_x x n_x, the couplings between rows are E = diag(e),
// e_i = -(hx/hz) (halved at i = 0, nx-1).
//
// Block LU with explicit Schur-complement inverses:
//     D_0 = A_0,  G_j = D_j^{-1},  D_{j+1} = A_{j+1} - E G_j E,
// forward sweep  w_j = G_j (b_j - E w_{j-1}),
// backward sweep x_j = w_j - G_j E x_{j+1}.
// G_j is computed in place by block Gauss-Jordan with pivoting inside each
// kb x kb diagonal tile: per panel K, T = (A_KK)^{-1} and
//     A <- A' + W V,  W = [-A_{:,K} T ; T - I],  V = [A_{K,:} with V_KK = I],
// A' = A with the K columns cleared (A'_KK = I).
// Blocks are padded to np = nx rounded up to 16 with an identity tail.
//
// Dense contractions (the rank-kb update and the sweeps) run on the matrix
// cores: v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32, complex products as
// four real products.  Lane l supplies A[l%16][k] and B[k][l%16] with the
// k index owned by lane group l/16; each lane loads four consecutive k of
// its row/column (64 contiguous bytes) and feeds them to four successive
// instructions, so every operand load is a contiguous vector load.
#include "helm_device.h"
#include "helm_launch.h"

namespace helm {
// ------------------------------------------------------ elementwise / FP64 --
__global__ void k_check_model(const double* m, int64_t n, int* flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        double v = m[i];
        if (!(v > 0.0) || !isfinite(v)) atomicOr(flag, 1);
    }
}

__global__ void k_zero(uint32_t* p, size_t n32) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n32) p[i] = 0u;
}

// r = B - A X (or A^*), FP64; per-block partial sums of |r|^2 and |B|^2
//
// A workgroup takes one block of 256 nodes and a group of RES_CS columns:
// each thread forms its node's stencil (the diagonal entry from m, the two
// couplings, the boundary cases) once and applies it to every column of the
// group.  All loads of all the group's columns are issued first, at clamped
// (in-range) addresses, and the boundary cases are applied afterwards, so
// none of them waits on another (with the neighbours loaded behind their
// boundary tests, every load was followed by its own wait).  Two columns
// per workgroup measured best at 401^2 (four and eight were slower).  The per-(column, block) partial sums keep
// one fixed order: a shuffle tree within each wavefront, then the four
// wavefront sums.
//
// Workgroups go to the eight XCDs in turn, so the (column group, block)
// pairs are numbered to give each XCD one contiguous range of them: the rows
// above and below a block, which the stencil reads, then belong to blocks
// on the same XCD and come from its L2 instead of being fetched again by
// every neighbour's XCD.  The grid has 8 * per_xcd workgroups; numbers past
// the nblk * ceil(S / RES_CS) pairs return at once.
constexpr int RES_CS = 2;

__global__ __launch_bounds__(256) void k_residual(Coef cf, int adjoint, const double2* __restrict__ B, int64_t ldb,
                                                  const double2* __restrict__ X, int64_t ldx,
                                                  double2* __restrict__ R, int64_t ldr, float2* __restrict__ R32,
                                                  int S, double* __restrict__ partial, int nblk, int per_xcd) {
    __shared__ double sr[RES_CS][4], sb[RES_CS][4];
    const int pair = (int)(blockIdx.x & 7u) * per_xcd + (int)(blockIdx.x >> 3);
    const int ncg = (S + RES_CS - 1) / RES_CS;
    if ((int64_t)pair >= (int64_t)nblk * ncg) return;
    const int cg = pair / nblk, kb = pair - cg * nblk;
    const int s0 = cg * RES_CS, ns = min(RES_CS, S - s0);
    const int nx = cf.nx, nz = cf.nz;
    const int N = nx * nz;                         // below 2^30 (grid check)
    const int k0 = kb * 256 + (int)threadIdx.x;
    const bool in = k0 < N;
    const int k = in ? k0 : N - 1;
    const int j = k / nx, i = k - j * nx;
    const bool hl = i > 0, hr = i < nx - 1, hu = j > 0, hd = j < nz - 1;
    const int kl = hl ? k - 1 : k, kr = hr ? k + 1 : k, ku = hu ? k - nx : k, kd = hd ? k + nx : k;
    double2 xc[RES_CS], xl[RES_CS], xr[RES_CS], xu[RES_CS], xd[RES_CS], bv[RES_CS];
#pragma unroll
    for (int c = 0; c < RES_CS; ++c) {
        const int s = s0 + min(c, ns - 1);
        const double2* x = X + (size_t)s * ldx;
        xc[c] = x[k];
        xl[c] = x[kl];
        xr[c] = x[kr];
        xu[c] = x[ku];
        xd[c] = x[kd];
        bv[c] = B[(size_t)s * ldb + k];
    }
    double2 dg = diag_entry(cf, i, j);
    if (adjoint) dg.y = -dg.y;
    const double cx = x_coupling(cf, j), cz = z_coupling(cf, i);
    double rr[RES_CS], bb[RES_CS];
#pragma unroll
    for (int c = 0; c < RES_CS; ++c) {
        rr[c] = 0.0;
        bb[c] = 0.0;
        if (in && c < ns) {
            const int s = s0 + c;
            double ar = dg.x * xc[c].x - dg.y * xc[c].y, ai = dg.x * xc[c].y + dg.y * xc[c].x;
            if (hl) { ar -= cx * xl[c].x; ai -= cx * xl[c].y; }
            if (hr) { ar -= cx * xr[c].x; ai -= cx * xr[c].y; }
            if (hu) { ar -= cz * xu[c].x; ai -= cz * xu[c].y; }
            if (hd) { ar -= cz * xd[c].x; ai -= cz * xd[c].y; }
            const double2 bk = bv[c];
            const double2 r = make_double2(bk.x - ar, bk.y - ai);
            if (R) R[(size_t)s * ldr + k] = r;
            if (R32) R32[(size_t)s * ldr + k] = make_float2((float)r.x, (float)(adjoint ? -r.y : r.y));
            rr[c] = r.x * r.x + r.y * r.y;
            bb[c] = bk.x * bk.x + bk.y * bk.y;
        }
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < RES_CS; ++c) {
        double a = rr[c], e = bb[c];
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_down(a, o, 64);
            e += __shfl_down(e, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            sr[c][w] = a;
            sb[c][w] = e;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < ns) {
        const int c = threadIdx.x;
        partial[((size_t)(s0 + c) * nblk + kb) * 2 + 0] = (sr[c][0] + sr[c][1]) + (sr[c][2] + sr[c][3]);
        partial[((size_t)(s0 + c) * nblk + kb) * 2 + 1] = (sb[c][0] + sb[c][1]) + (sb[c][2] + sb[c][3]);
    }
}

// per column s: the sums of the per-block partials, one workgroup per
// column, strided partial sums then a fixed-order tree in LDS
__global__ __launch_bounds__(256) void k_norms_finish(const double* partial, int nblk, int S, double* norms) {
    __shared__ double sa[256], sc[256];
    const int s = blockIdx.x, t = threadIdx.x;
    double a = 0.0, c = 0.0;
    for (int q = t; q < nblk; q += 256) {
        a += partial[((size_t)s * nblk + q) * 2];
        c += partial[((size_t)s * nblk + q) * 2 + 1];
    }
    sa[t] = a;
    sc[t] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            sa[t] += sa[t + h];
            sc[t] += sc[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        norms[2 * s] = sa[0];
        norms[2 * s + 1] = sc[0];
    }
}

__global__ void k_c128_to_c64(const double2* src, int64_t lds, float2* dst, int64_t ldd, int64_t N, int conj) {
    const int s = blockIdx.y;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    double2 v = src[(size_t)s * lds + k];
    dst[(size_t)s * ldd + k] = make_float2((float)v.x, (float)(conj ? -v.y : v.y));
}

__global__ void k_c64_to_c128(const float2* src, int64_t lds, double2* dst, int64_t ldd, int64_t N, int conj,
                              int accumulate) {
    const int s = blockIdx.y;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    float2 v = src[(size_t)s * lds + k];
    double re = v.x, im = conj ? -(double)v.y : (double)v.y;
    double2* o = dst + (size_t)s * ldd + k;
    if (accumulate) { double2 p = *o; *o = make_double2(p.x + re, p.y + im); }
    else *o = make_double2(re, im);
}

__global__ void k_conj(double2* X, int64_t ld, int64_t N) {
    const int s = blockIdx.y;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N) X[(size_t)s * ld + k].y = -X[(size_t)s * ld + k].y;
}

__global__ void k_axpy(const double2* D, int64_t ldd, double2* X, int64_t ldx, int64_t N) {
    const int s = blockIdx.y;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    double2 a = D[(size_t)s * ldd + k], x = X[(size_t)s * ldx + k];
    X[(size_t)s * ldx + k] = make_double2(x.x + a.x, x.y + a.y);
}

__global__ void k_unit_sources(double2* E, int64_t ld, int64_t N, const int* nodes) {
    const int s = blockIdx.y;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < N) E[(size_t)s * ld + k] = make_double2(k == nodes[s] ? 1.0 : 0.0, 0.0);
}

// boundary weight b_k: half the length of each boundary edge at node k
__device__ __forceinline__ double bnd_weight(const Coef& c, int i, int j) {
    double bnd = 0.0;
    if (j == 0 || j == c.nz - 1) bnd += 0.5 * c.hx * ((i > 0 ? 1 : 0) + (i < c.nx - 1 ? 1 : 0));
    if (i == 0 || i == c.nx - 1) bnd += 0.5 * c.hz * ((j > 0 ? 1 : 0) + (j < c.nz - 1 ? 1 : 0));
    return bnd;
}

// nodal weight of G_{m,w}(beta_k .): w^2 d_k + b_k i w / (2 sqrt m_k)
__device__ __forceinline__ double2 grad_weight(const Coef& c, int i, int j) {
    double mass = c.hx * c.hz * half_at_ends(i, c.nx) * half_at_ends(j, c.nz);
    double mk_ = c.m[(size_t)j * c.nx + i];
    return make_double2(c.omega * c.omega * mass, c.omega * bnd_weight(c, i, j) / (2.0 * sqrt(mk_)));
}

// g_k += -Re sum_s wk u_{s,k} conj(l_{s,k})
__global__ __launch_bounds__(256) void k_grad(Coef cf, const double2* U, int64_t ldu, const double2* L,
                                              int64_t ldl, int S, double* g) {
    const int64_t N = (int64_t)cf.nx * cf.nz;
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    double2 wk = grad_weight(cf, (int)(k % cf.nx), (int)(k / cf.nx));
    double sr = 0.0, si = 0.0;   // sum_s u conj(l)
    for (int s = 0; s < S; ++s) {
        double2 u = U[(size_t)s * ldu + k], l = L[(size_t)s * ldl + k];
        sr += u.x * l.x + u.y * l.y;
        si += u.y * l.x - u.x * l.y;
    }
    g[k] += -(wk.x * sr - wk.y * si);
}

// V[(a*S + s)] = wk * mt_a[k] * u_s[k]
__global__ void k_gn_rhs(Coef cf, const double2* U, int64_t ldu, int S, const double* mt, int n_dir,
                         double2* V, int64_t ldv) {
    const int64_t N = (int64_t)cf.nx * cf.nz;
    const int col = blockIdx.y;   // a*S + s
    const int a = col / S, s = col % S;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    double2 wk = grad_weight(cf, (int)(k % cf.nx), (int)(k / cf.nx));
    double2 u = U[(size_t)s * ldu + k];
    double t = mt[(size_t)a * N + k];
    V[(size_t)col * ldv + k] = make_double2(t * (wk.x * u.x - wk.y * u.y), t * (wk.x * u.y + wk.y * u.x));
}

// hv_a[k] += Re sum_s wk u_s[k] conj(z_{a,s}[k])
__global__ void k_hv(Coef cf, const double2* U, int64_t ldu, int S, const double2* Z, int64_t ldz, int n_dir,
                     double* hv) {
    const int64_t N = (int64_t)cf.nx * cf.nz;
    const int a = blockIdx.y;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    double2 wk = grad_weight(cf, (int)(k % cf.nx), (int)(k / cf.nx));
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < S; ++s) {
        double2 u = U[(size_t)s * ldu + k], z = Z[(size_t)(a * S + s) * ldz + k];
        sr += u.x * z.x + u.y * z.y;
        si += u.y * z.x - u.x * z.y;
    }
    hv[(size_t)a * N + k] += wk.x * sr - wk.y * si;
}

// Point sources between nodes: column q of E (zeroed beforehand) receives
// phi_j(s_q), the P1 hat functions of the rectangles cut into triangles,
// averaged over the two ways of cutting (at a node: e_s).  One thread per
// source, so no two threads write one column.
__global__ void k_point_sources(double2* E, int64_t ld, const double* xz, int S, int nx, int nz, double hx,
                                double hz) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= S) return;
    const double u = xz[2 * q] / hx, v = xz[2 * q + 1] / hz;
    const int i = min((int)floor(u), nx - 2), j = min((int)floor(v), nz - 2);
    const double xi = u - i, eta = v - j;
    double w00 = 0.0, w10 = 0.0, w01 = 0.0, w11 = 0.0;
    if (xi >= eta) {   // cut (i, j)-(i+1, j+1), lower triangle
        w00 += 1.0 - xi, w10 += xi - eta, w11 += eta;
    } else {
        w00 += 1.0 - eta, w01 += eta - xi, w11 += xi;
    }
    if (xi + eta <= 1.0) {   // cut (i+1, j)-(i, j+1)
        w00 += 1.0 - xi - eta, w10 += xi, w01 += eta;
    } else {
        w11 += xi + eta - 1.0, w10 += 1.0 - eta, w01 += 1.0 - xi;
    }
    double2* col = E + (size_t)q * ld;
    const int64_t k00 = (int64_t)j * nx + i;
    col[k00] = make_double2(0.5 * w00, 0.0);
    col[k00 + 1] = make_double2(0.5 * w10, 0.0);
    col[k00 + nx] = make_double2(0.5 * w01, 0.0);
    col[k00 + nx + 1] = make_double2(0.5 * w11, 0.0);
}

// ---- restriction R(P): per sensor q up to RTAP taps (node[q*RTAP + a],
// weight w[q*RTAP + a]); ntap = 1 for sensors on nodes, 16 for the sliding
// bicubic of sensors between nodes.  w may be the value weights or those of
// a derivative with respect to the sensor's coordinates.

// out[c][q] = sum_a w[q][a] U[c][node[q][a]]
__global__ void k_restrict(const double2* U, int64_t ldu, const int* node, const double* w, int ntap, int Nr,
                           double2* out, int64_t ldo) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (q >= Nr) return;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < ntap; ++a) {
        const double wa = w[q * RTAP + a];
        const double2 u = U[(size_t)c * ldu + node[q * RTAP + a]];
        re += wa * u.x;
        im += wa * u.y;
    }
    out[(size_t)c * ldo + q] = make_double2(re, im);
}

// eps_s = d_s - R u_s and 1/2 |eps_s|^2: one block of 64 threads per
// source, the sensors strided over the threads, |eps|^2 summed in a fixed order
__global__ __launch_bounds__(64) void k_misfit(const double2* U, int64_t ldu, const double2* dobs, const int* node,
                                               const double* w, int ntap, int Nr, double2* eps, double* phi_part) {
    __shared__ double sq[64];
    const int s = blockIdx.x;
    double acc = 0.0;
    for (int q = threadIdx.x; q < Nr; q += 64) {
        double re = 0.0, im = 0.0;
        for (int a = 0; a < ntap; ++a) {
            const double wa = w[q * RTAP + a];
            const double2 u = U[(size_t)s * ldu + node[q * RTAP + a]];
            re += wa * u.x;
            im += wa * u.y;
        }
        double2 dv = dobs[(size_t)s * Nr + q];
        double2 e = make_double2(dv.x - re, dv.y - im);
        eps[(size_t)s * Nr + q] = e;
        acc += e.x * e.x + e.y * e.y;
    }
    sq[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sq[threadIdx.x] += sq[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) phi_part[s] = 0.5 * sq[0];
}

// out[c][tnode[t]] += sum_{e in row t} tw[e] Z[c][tq[e]]: R^T z gathered per
// distinct node (the transpose of the taps), so no two threads write one element
__global__ void k_restrict_adj(const double2* Z, int64_t ldz, const int* tnode, const int* tptr, const int* tq,
                               const double* tw, int nt, double2* out, int64_t ldo) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (t >= nt) return;
    double re = 0.0, im = 0.0;
    for (int e = tptr[t]; e < tptr[t + 1]; ++e) {
        const double2 z = Z[(size_t)c * ldz + tq[e]];
        re += tw[e] * z.x;
        im += tw[e] * z.y;
    }
    double2* o = out + (size_t)c * ldo + tnode[t];
    *o = make_double2(o->x + re, o->y + im);
}

// Upper-level derivative, one frequency (one block of 64 threads per sensor q,
// the sources strided over the threads, summed in a fixed order):
//   dp[q][l] += -sum_s Re[ (d_l tau)(p_q) conj(eps_sq) + tau(p_q) conj(dd_sql - (d_l u)(p_q)) ]
// eps = R(u' - u) (the misfit), dd = dR/dx_l u' (the training data's derivative)
__global__ __launch_bounds__(64) void k_upper(const double2* Tau, const double2* U, int64_t ld, int S,
                                              const double2* eps, const double2* dd, const int* node,
                                              const double* w0, const double* wx, const double* wz, int Nr,
                                              double* dp) {
    __shared__ double sx[64], sz[64];
    const int q = blockIdx.x;
    double ax = 0.0, az = 0.0;
    for (int s = threadIdx.x; s < S; s += 64) {
        double2 t0 = make_double2(0.0, 0.0), tx = t0, tz = t0, ux = t0, uz = t0;
        for (int a = 0; a < RTAP; ++a) {
            const int k = node[q * RTAP + a];
            const double v0 = w0[q * RTAP + a], vx = wx[q * RTAP + a], vz = wz[q * RTAP + a];
            const double2 tv = Tau[(size_t)s * ld + k], uv = U[(size_t)s * ld + k];
            t0.x += v0 * tv.x; t0.y += v0 * tv.y;
            tx.x += vx * tv.x; tx.y += vx * tv.y;
            tz.x += vz * tv.x; tz.y += vz * tv.y;
            ux.x += vx * uv.x; ux.y += vx * uv.y;
            uz.x += vz * uv.x; uz.y += vz * uv.y;
        }
        const double2 e = eps[(size_t)s * Nr + q];
        const double2 gx = dd[((size_t)s * Nr + q) * 2 + 0], gz = dd[((size_t)s * Nr + q) * 2 + 1];
        const double2 fx = make_double2(gx.x - ux.x, gx.y - ux.y), fz = make_double2(gz.x - uz.x, gz.y - uz.y);
        // Re[a conj(b)] = a.x b.x + a.y b.y
        ax -= tx.x * e.x + tx.y * e.y + t0.x * fx.x + t0.y * fx.y;
        az -= tz.x * e.x + tz.y * e.y + t0.x * fz.x + t0.y * fz.y;
    }
    sx[threadIdx.x] = ax;
    sz[threadIdx.x] = az;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sx[threadIdx.x] += sx[threadIdx.x + h];
            sz[threadIdx.x] += sz[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dp[2 * q] += sx[0];
        dp[2 * q + 1] += sz[0];
    }
}

// W[(a*S + s)] = -conj(wk) * mt_a[k] * l_s[k]: the second-order part of the
// right-hand side of the last adjoint solve of a Hessian product (the
// receiver part R^* R v is added onto it afterwards)
__global__ void k_zeta_rhs(Coef cf, const double2* L, int64_t ldl, int S, const double* mt, double2* W,
                           int64_t ldw) {
    const int64_t N = (int64_t)cf.nx * cf.nz;
    const int col = blockIdx.y;
    const int a = col / S, s = col % S;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    double2 wk = grad_weight(cf, (int)(k % cf.nx), (int)(k / cf.nx));
    double2 l = L[(size_t)s * ldl + k];
    double t = mt[(size_t)a * N + k];
    // -(wr - i wi)(lr + i li) t
    W[(size_t)col * ldw + k] = make_double2(-t * (wk.x * l.x + wk.y * l.y), -t * (wk.x * l.y - wk.y * l.x));
}

// Full Hessian product, one frequency:
// hv_a[k] += Re wk sum_s (u conj z - v conj l) - mt_a[k] Re hk sum_s u conj l,
// hk = d wk / d m_k = -i w b_k / (4 m_k^{3/2})
__global__ __launch_bounds__(256) void k_hv_full(Coef cf, const double2* U, const double2* L, int64_t ldu, int S,
                                                 const double2* V, const double2* Z, int64_t ldz, const double* mt,
                                                 double* hv) {
    const int64_t N = (int64_t)cf.nx * cf.nz;
    const int a = blockIdx.y;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int i = (int)(k % cf.nx), j = (int)(k / cf.nx);
    double2 wk = grad_weight(cf, i, j);
    double ar = 0.0, ai = 0.0;   // sum_s u conj z - v conj l
    double pi = 0.0;             // Im sum_s u conj l
    for (int s = 0; s < S; ++s) {
        const size_t o = (size_t)s * ldu + k, oz = (size_t)(a * S + s) * ldz + k;
        double2 u = U[o], l = L[o], v = V[oz], z = Z[oz];
        ar += u.x * z.x + u.y * z.y - (v.x * l.x + v.y * l.y);
        ai += u.y * z.x - u.x * z.y - (v.y * l.x - v.x * l.y);
        pi += u.y * l.x - u.x * l.y;
    }
    const double mk_ = cf.m[k];
    const double hi = -cf.omega * bnd_weight(cf, i, j) / (4.0 * mk_ * sqrt(mk_));   // hk = i hi
    hv[(size_t)a * N + k] += (wk.x * ar - wk.y * ai) + mt[(size_t)a * N + k] * hi * pi;
}

// partial sums of x . y, one per 256-thread block
__global__ __launch_bounds__(256) void k_dot(const double* x, const double* y, int64_t n, double* part) {
    __shared__ double sq[256];
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    sq[threadIdx.x] = k < n ? x[k] * y[k] : 0.0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sq[threadIdx.x] += sq[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sq[0];
}

// per-block maxima of |x|
__global__ __launch_bounds__(256) void k_absmax(const double* x, int64_t n, double* part) {
    __shared__ double sq[256];
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    sq[threadIdx.x] = k < n ? fabs(x[k]) : 0.0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sq[threadIdx.x] = fmax(sq[threadIdx.x], sq[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sq[0];
}

// out = a x + b y (out may be x or y)
__global__ void k_lincomb(double* out, double a, const double* x, double b, const double* y, int64_t n) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = a * x[k] + b * y[k];
}

// g += Gamma m and partial sums of m^T Gamma m, Gamma = alpha (Dx^T Dx + Dz^T Dz) + mu I,
// D_n = (n - 1) bidiag(1, -1)
__global__ __launch_bounds__(256) void k_gamma(const double* m, int nx, int nz, double alpha, double mu,
                                               double* g, double* part) {
    __shared__ double sq[256];
    const int64_t N = (int64_t)nx * nz;
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double q = 0.0;
    if (k < N) {
        const int i = (int)(k % nx), j = (int)(k / nx);
        const double ax = (double)(nx - 1) * (nx - 1), az = (double)(nz - 1) * (nz - 1);
        double mk_ = m[k], rm = 0.0;
        if (i > 0) rm += ax * (mk_ - m[k - 1]);
        if (i < nx - 1) rm += ax * (mk_ - m[k + 1]);
        if (j > 0) rm += az * (mk_ - m[k - nx]);
        if (j < nz - 1) rm += az * (mk_ - m[k + nx]);
        double gm = alpha * rm + mu * mk_;
        g[k] += gm;
        q = mk_ * gm;
    }
    sq[threadIdx.x] = q;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sq[threadIdx.x] += sq[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sq[0];
}

// sum of n partials by one wavefront (64 threads): lane l adds part[l],
// part[l + 64], ... in order, then a fixed-order tree across the lanes
__global__ void k_sum_scalar(const double* part, int n, double* out) {
    const int l = threadIdx.x;
    double a = 0.0;
    for (int q = l; q < n; q += 64) a += part[q];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
    if (l == 0) *out = a;
}

// one wavefront: D = A(16x4) B(4x16) with the operand layout the kernels assume
__global__ void k_mfma_probe(int prec, const double* A, const double* B, double* D) {
    const int l = threadIdx.x;
    if (prec == 0) {
        v4d c = {0, 0, 0, 0};
        c = mfma16(A[(l % 16) * 4 + l / 16], B[(l / 16) * 16 + l % 16], c);
#pragma unroll
        for (int e = 0; e < 4; ++e) D[acc_row<double>(l / 16, e) * 16 + l % 16] = c[e];
    } else {
        v4f c = {0, 0, 0, 0};
        c = mfma16((float)A[(l % 16) * 4 + l / 16], (float)B[(l / 16) * 16 + l % 16], c);
#pragma unroll
        for (int e = 0; e < 4; ++e) D[acc_row<float>(l / 16, e) * 16 + l % 16] = (double)c[e];
    }
}

// ---------------------------------------------------------------- launchers --
static inline dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

// A group's front table into device memory (one workgroup, one dword per
// thread), in stream order before the group's launches.
template <typename Tab>
__global__ __launch_bounds__(256) void k_put_table(const Tab src, Tab* dst) {
    static_assert(sizeof(Tab) % 4 == 0, "tables are whole dwords");
    constexpr int W = (int)(sizeof(Tab) / 4);
    const uint32_t* s = (const uint32_t*)&src;
    uint32_t* d = (uint32_t*)dst;
    for (int i = threadIdx.x; i < W; i += 256) d[i] = s[i];
}
void launch_put_chain_table(const ChainTab& tab, ChainTab* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_put_table<ChainTab>, dim3(1), dim3(256), 0, st, tab, dst);
}
void launch_put_sweep_table(const SweepTab& tab, SweepTab* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_put_table<SweepTab>, dim3(1), dim3(256), 0, st, tab, dst);
}

void launch_check_model(const double* m, int64_t n, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_check_model, grid1(n), dim3(256), 0, st, m, n, flag);
}
void launch_residual(const Coef& cf, int adjoint, const double* B, int64_t ldb, const double* X, int64_t ldx,
                     double* R, int64_t ldr, float* R32, int S, double* partial, int nblk, hipStream_t st) {
    const int per_xcd = (int)(((int64_t)nblk * ((S + RES_CS - 1) / RES_CS) + 7) / 8);
    hipLaunchKernelGGL(k_residual, dim3(8 * per_xcd), dim3(256), 0, st, cf, adjoint, (const double2*)B, ldb,
                       (const double2*)X, ldx, (double2*)R, ldr, (float2*)R32, S, partial, nblk, per_xcd);
}
void launch_norms_finish(const double* partial, int nblk, int S, double* norms, hipStream_t st) {
    hipLaunchKernelGGL(k_norms_finish, dim3(S), dim3(256), 0, st, partial, nblk, S, norms);
}
void launch_c128_to_c64(const double* src, int64_t lds, float* dst, int64_t ldd, int64_t N, int S, int conj,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_c128_to_c64, dim3(grid1(N).x, S), dim3(256), 0, st, (const double2*)src, lds,
                       (float2*)dst, ldd, N, conj);
}
void launch_c64_to_c128(const float* src, int64_t lds, double* dst, int64_t ldd, int64_t N, int S, int conj,
                        int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_c64_to_c128, dim3(grid1(N).x, S), dim3(256), 0, st, (const float2*)src, lds,
                       (double2*)dst, ldd, N, conj, accumulate);
}
void launch_conj_inplace(double* X, int64_t ld, int64_t N, int S, hipStream_t st) {
    hipLaunchKernelGGL(k_conj, dim3(grid1(N).x, S), dim3(256), 0, st, (double2*)X, ld, N);
}
void launch_axpy_c128(const double* D, int64_t ldd, double* X, int64_t ldx, int64_t N, int S, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy, dim3(grid1(N).x, S), dim3(256), 0, st, (const double2*)D, ldd, (double2*)X, ldx, N);
}
void launch_unit_sources(double* E, int64_t ld, int64_t N, const int* nodes, int S, hipStream_t st) {
    hipLaunchKernelGGL(k_unit_sources, dim3(grid1(N).x, S), dim3(256), 0, st, (double2*)E, ld, N, nodes);
}
void launch_misfit(const double* U, int64_t ldu, const double* dobs, const int* node, const double* w, int ntap,
                   int Nr, int S, double* eps, double* phi_part, hipStream_t st) {
    hipLaunchKernelGGL(k_misfit, dim3(S), dim3(64), 0, st, (const double2*)U, ldu, (const double2*)dobs, node, w,
                       ntap, Nr, (double2*)eps, phi_part);
}
void launch_point_sources(double* E, int64_t ld, const double* xz, int S, int nx, int nz, double hx, double hz,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_point_sources, grid1(S, 64), dim3(64), 0, st, (double2*)E, ld, xz, S, nx, nz, hx, hz);
}
void launch_restrict(const double* U, int64_t ldu, const int* node, const double* w, int ntap, int Nr, int cols,
                     double* out, int64_t ldo, hipStream_t st) {
    hipLaunchKernelGGL(k_restrict, dim3(grid1(Nr, 64).x, cols), dim3(64), 0, st, (const double2*)U, ldu, node, w, ntap,
                       Nr, (double2*)out, ldo);
}
void launch_restrict_adj(const double* Z, int64_t ldz, const int* tnode, const int* tptr, const int* tq,
                         const double* tw, int nt, int cols, double* out, int64_t ldo, hipStream_t st) {
    hipLaunchKernelGGL(k_restrict_adj, dim3(grid1(nt, 64).x, cols), dim3(64), 0, st, (const double2*)Z, ldz, tnode,
                       tptr, tq, tw, nt, (double2*)out, ldo);
}
void launch_upper(const double* Tau, const double* U, int64_t ld, int S, const double* eps, const double* dd,
                  const int* node, const double* w0, const double* wx, const double* wz, int Nr, double* dp,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_upper, dim3(Nr), dim3(64), 0, st, (const double2*)Tau, (const double2*)U, ld, S,
                       (const double2*)eps, (const double2*)dd, node, w0, wx, wz, Nr, dp);
}
void launch_grad(const Coef& cf, const double* U, int64_t ldu, const double* L, int64_t ldl, int S, double* g,
                 hipStream_t st) {
    hipLaunchKernelGGL(k_grad, grid1((int64_t)cf.nx * cf.nz), dim3(256), 0, st, cf, (const double2*)U, ldu,
                       (const double2*)L, ldl, S, g);
}
void launch_gn_rhs(const Coef& cf, const double* U, int64_t ldu, int S, const double* mt, int n_dir, double* V,
                   int64_t ldv, hipStream_t st) {
    hipLaunchKernelGGL(k_gn_rhs, dim3(grid1((int64_t)cf.nx * cf.nz).x, n_dir * S), dim3(256), 0, st, cf,
                       (const double2*)U, ldu, S, mt, n_dir, (double2*)V, ldv);
}
void launch_hv(const Coef& cf, const double* U, int64_t ldu, int S, const double* Z, int64_t ldz, int n_dir,
               double* hv, int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_hv, dim3(grid1(N).x, n_dir), dim3(256), 0, st, cf, (const double2*)U, ldu, S,
                       (const double2*)Z, ldz, n_dir, hv);
}
void launch_zeta_rhs(const Coef& cf, const double* L, int64_t ldl, int S, const double* mt, int n_dir, double* W,
                     int64_t ldw, hipStream_t st) {
    hipLaunchKernelGGL(k_zeta_rhs, dim3(grid1((int64_t)cf.nx * cf.nz).x, n_dir * S), dim3(256), 0, st, cf,
                       (const double2*)L, ldl, S, mt, (double2*)W, ldw);
}
void launch_hv_full(const Coef& cf, const double* U, const double* L, int64_t ldu, int S, const double* V,
                    const double* Z, int64_t ldz, const double* mt, int n_dir, double* hv, hipStream_t st) {
    hipLaunchKernelGGL(k_hv_full, dim3(grid1((int64_t)cf.nx * cf.nz).x, n_dir), dim3(256), 0, st, cf,
                       (const double2*)U, (const double2*)L, ldu, S, (const double2*)V, (const double2*)Z, ldz, mt,
                       hv);
}
int dot_blocks(int64_t n) { return (int)((n + 255) / 256); }
void launch_dot(const double* x, const double* y, int64_t n, double* part, double* out, hipStream_t st) {
    const int nb = dot_blocks(n);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(256), 0, st, x, y, n, part);
    hipLaunchKernelGGL(k_sum_scalar, dim3(1), dim3(64), 0, st, part, nb, out);
}
void launch_absmax(const double* x, int64_t n, double* part, hipStream_t st) {
    hipLaunchKernelGGL(k_absmax, dim3(dot_blocks(n)), dim3(256), 0, st, x, n, part);
}
void launch_lincomb(double* out, double a, const double* x, double b, const double* y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_lincomb, grid1(n), dim3(256), 0, st, out, a, x, b, y, n);
}
void launch_gamma(const double* m, int nx, int nz, double alpha, double mu, double* g, double* part, int nblk,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_gamma, dim3(nblk), dim3(256), 0, st, m, nx, nz, alpha, mu, g, part);
}
void launch_sum_scalar(const double* part, int n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_scalar, dim3(1), dim3(64), 0, st, part, n, out);
}
void launch_zero(void* p, size_t bytes, hipStream_t st) {
    size_t n32 = (bytes + 3) / 4;
    if (n32) hipLaunchKernelGGL(k_zero, grid1((int64_t)n32), dim3(256), 0, st, (uint32_t*)p, n32);
}
void launch_mfma_probe(int prec, const double* A, const double* B, double* D, hipStream_t st) {
    hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, st, prec, A, B, D);
}

}  // namespace helm
