// Block factorisation kernels of libhelm (gfx950).
//
// For each system the Schur complements of the block-tridiagonal operator,
//     D_0 = A_0,   D_{j+1} = A_{j+1} - E D_j^{-1} E,
// are inverted in place by block Gauss-Jordan on panels of KB = 32 columns.
// Panel K of block j, with T = (X_KK)^{-1} the inverse of its diagonal tile
// (pivoting inside the tile only), maps the working block X to
//     Y = X' + W V,   W = [-X_{:,K} T ; T - I],   V = [X_{K,:} with V_KK = I],
// X' = X with the K columns cleared except X'_KK = I.  After the last panel Y
// is D_j^{-1}; the same launch also writes D_{j+1} for the next block.
//
// One launch per panel step serves every chain of the batch.  Its
// workgroups are the 64 x 64 output tiles of Y (each forms its rows of W
// from X and T itself, so X and Y live in different buffers and no copy of
// V is needed) plus one workgroup per chain that builds the diagonal tile
// the NEXT step needs,
//     Z = X_{K'K'} - X_{K'K} T X_{KK'}            (next panel K' of block j), or
//     Z = A_{j+1}[K'K'] - E (Y restricted) E       (first panel of block j+1),
// and inverts it, so the sequential pivoting of the next step runs
// concurrently with this step's matrix-core update.
#include "helm_device.h"
#include "helm_launch.h"

namespace helm {

// --------------------------------------------------- diagonal-tile inverse --
// Gauss-Jordan inversion of a kb x kb tile (kb = 16 or 32) by 256 threads:
// thread t holds row r = t/8 (wave w = t/64 holds rows 8w..8w+7) and columns
// 4(t%8) .. 4(t%8)+3.  Partial pivoting over the unused rows of the tile.
// Each wave nominates its best candidate row for the next column (key =
// magnitude bits with the row index in the low bits, reduced with DPP) and
// publishes it with the row's values; one barrier per pivot.  Rows are not
// moved: the pivot of column p sits in row rowOf[p], and the inverse is
// T[i][c] = M[rowOf[i]][stepOf[c]].

template <typename T>
struct GJScratch {
    uint32_t key[2][4];
    typename CT<T>::c row[2][4][32];
    int rowOf[32];
    int stepOf[32];
};

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row half-mirror
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row mirror
    const uint32_t a = __builtin_amdgcn_readlane((int)v, 0), b = __builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = __builtin_amdgcn_readlane((int)v, 32), d = __builtin_amdgcn_readlane((int)v, 48);
    return max(max(a, b), max(c, d));
}

// value held by lane (l & ~7) | src within each group of 32 lanes
template <int SRC>
__device__ __forceinline__ int swz_row(int v) {
    return __builtin_amdgcn_ds_swizzle(v, 0x18 | (SRC << 5));
}
template <int SRC>
__device__ __forceinline__ double swz_row(double v) {
    const int lo = swz_row<SRC>(__double2loint(v)), hi = swz_row<SRC>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int SRC>
__device__ __forceinline__ float swz_row(float v) {
    return __int_as_float(swz_row<SRC>(__float_as_int(v)));
}
template <typename T>
__device__ __forceinline__ typename CT<T>::c swz_row_c(typename CT<T>::c v, int src) {
    using C = typename CT<T>::c;
    C r;
    switch (src) {
#define HELM_SWZ(k) case k: r.x = swz_row<k>(v.x); r.y = swz_row<k>(v.y); break;
        HELM_SWZ(0) HELM_SWZ(1) HELM_SWZ(2) HELM_SWZ(3) HELM_SWZ(4) HELM_SWZ(5) HELM_SWZ(6)
        default: r.x = swz_row<7>(v.x); r.y = swz_row<7>(v.y); break;
#undef HELM_SWZ
    }
    return r;
}

// 1 / p for complex p, reciprocal of |p|^2 refined by Newton steps
__device__ __forceinline__ double2 crcp(double2 p) {
    const double n = p.x * p.x + p.y * p.y;
    double y = __builtin_amdgcn_rcp(n);
    y = y * (2.0 - n * y);
    y = y * (2.0 - n * y);
    return make_double2(p.x * y, -p.y * y);
}
__device__ __forceinline__ float2 crcp(float2 p) {
    const float n = p.x * p.x + p.y * p.y;
    float y = __builtin_amdgcn_rcpf(n);
    y = y * (2.0f - n * y);
    return make_float2(p.x * y, -p.y * y);
}

template <typename T>
__device__ __forceinline__ uint32_t pivot_key(typename CT<T>::c v, int r, bool cand) {
    if (!cand) return 0u;
    const float mag = (float)(v.x * v.x + v.y * v.y);
    return (__float_as_uint(mag) & ~0x3Fu) | 0x20u | (uint32_t)(31 - r);
}

// Inverts the tile held in a[] (layout above); on return a[] holds M and
// sh.rowOf / sh.stepOf the pivot order (valid after a barrier).  Returns the
// first pivot step whose candidates were all zero, or -1.
template <typename T, int KBT>
__device__ __forceinline__ int gj_invert(typename CT<T>::c (&a)[4], GJScratch<T>& sh) {
    using C = typename CT<T>::c;
    constexpr int NW = KBT / 8;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int r = t >> 3, cg = t & 7;
    const bool act = (r < KBT) && (4 * cg < KBT);
    uint32_t used = 0u;
    int zero = -1;
    {
        const uint32_t k = pivot_key<T>(a[0], r, act && cg == 0);
        const uint32_t wk = wave_max_u32(k);
        if (w < NW) {
            if (act && wk != 0u && r == 31 - (int)(wk & 31u)) {
#pragma unroll
                for (int e = 0; e < 4; ++e) sh.row[0][w][4 * cg + e] = a[e];
            }
            if (l == 0) sh.key[0][w] = wk;
        }
    }
#pragma unroll
    for (int p = 0; p < KBT; ++p) {
        const int par = p & 1;
        const int pc = p >> 2, pe = p & 3;
        __syncthreads();
        uint32_t best = sh.key[par][0];
        int wb = 0;
#pragma unroll
        for (int q = 1; q < NW; ++q) {
            const uint32_t kq = sh.key[par][q];
            if (kq > best) { best = kq; wb = q; }
        }
        const int rp = 31 - (int)(best & 31u);
        const bool good = (best >> 6) != 0u;
        if (!good && zero < 0) zero = p;
        const C piv = sh.row[par][wb][p];
        C pr[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) pr[e] = sh.row[par][wb][4 * cg + e];
        const C f = swz_row_c<T>(a[pe], pc);
        const C dv = HELM_CSEL(good, crcp(piv), mk<C>(0.0, 0.0));
        if (act) {
            if (r == rp) {
#pragma unroll
                for (int e = 0; e < 4; ++e) a[e] = (4 * cg + e == p) ? dv : cmul(pr[e], dv);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (4 * cg + e == p) {
                        a[e] = mk<C>(-(f.x * dv.x - f.y * dv.y), -(f.x * dv.y + f.y * dv.x));
                    } else {
                        const C s = cmul(pr[e], dv);
                        a[e] = mk<C>(a[e].x - (f.x * s.x - f.y * s.y), a[e].y - (f.x * s.y + f.y * s.x));
                    }
                }
            }
        }
        used |= 1u << rp;
        if (t == 0) { sh.rowOf[p] = rp; sh.stepOf[rp] = p; }
        if (p + 1 < KBT) {
            const int pc1 = (p + 1) >> 2, pe1 = (p + 1) & 3;
            const uint32_t k = pivot_key<T>(a[pe1], r, act && cg == pc1 && !((used >> r) & 1u));
            const uint32_t wk = wave_max_u32(k);
            if (w < NW) {
                if (act && wk != 0u && r == 31 - (int)(wk & 31u)) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) sh.row[par ^ 1][w][4 * cg + e] = a[e];
                }
                if (l == 0) sh.key[par ^ 1][w] = wk;
            }
        }
    }
    return zero;
}

// Scratch of the unpivoted inverses: the tile maximum of each wavefront and
// the small-pivot flag.
template <typename T>
struct RowScratch {
    float amax[4];
    int small;
};

// ------------------------------------------------ blocked unpivoted inverse --
// The diagonal tile [[A, B], [C, D]] (16 x 16 quadrants) is inverted as
//     A^-1,  X = A^-1 B,  Y = C A^-1,  S = D - Y B,  S^-1,
//     T12 = -X S^-1,  T21 = -S^-1 Y,  T22 = S^-1,  T11 = A^-1 - X T21,
// which is unpivoted Gauss-Jordan on the whole tile with its pivots taken in
// the same order (those of A, then those of S), so the small-pivot test is
// the same one.  The two 16 x 16 inverses are done by one wavefront each in
// registers (lane l holds row l % 16, columns 4 (l / 16) .. +3), exchanging
// the pivot row and column by cross-lane reads, with no barrier; the six
// 16 x 16 products run on the matrix cores from LDS.

template <typename C> __device__ __forceinline__ C lane_read(C v, int lane);
template <> __device__ __forceinline__ float2 lane_read(float2 v, int lane) {
    float2 r;
    r.x = __int_as_float(__builtin_amdgcn_ds_bpermute(lane << 2, __float_as_int(v.x)));
    r.y = __int_as_float(__builtin_amdgcn_ds_bpermute(lane << 2, __float_as_int(v.y)));
    return r;
}
template <> __device__ __forceinline__ double2 lane_read(double2 v, int lane) {
    const int a = lane << 2;
    const int xl = __builtin_amdgcn_ds_bpermute(a, __double2loint(v.x));
    const int xh = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v.x));
    const int yl = __builtin_amdgcn_ds_bpermute(a, __double2loint(v.y));
    const int yh = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v.y));
    return make_double2(__hiloint2double(xh, xl), __hiloint2double(yh, yl));
}
// the value of lane `lane` in every lane (lane is wave-uniform)
template <typename C> __device__ __forceinline__ C lane_bcast(C v, int lane);
template <> __device__ __forceinline__ float2 lane_bcast(float2 v, int lane) {
    return make_float2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), lane)),
                       __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), lane)));
}
template <> __device__ __forceinline__ double2 lane_bcast(double2 v, int lane) {
    const int xl = __builtin_amdgcn_readlane(__double2loint(v.x), lane);
    const int xh = __builtin_amdgcn_readlane(__double2hiint(v.x), lane);
    const int yl = __builtin_amdgcn_readlane(__double2loint(v.y), lane);
    const int yh = __builtin_amdgcn_readlane(__double2hiint(v.y), lane);
    return make_double2(__hiloint2double(xh, xl), __hiloint2double(yh, yl));
}

// the value of lane P of each row of 16 lanes, in every lane of that row
// (DPP row broadcast; P compile-time)
template <int P> __device__ __forceinline__ int row_bcast_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x150 + P, 0xF, 0xF, false);
}
template <int P> __device__ __forceinline__ float2 row_bcast(float2 v) {
    return make_float2(__int_as_float(row_bcast_i<P>(__float_as_int(v.x))),
                       __int_as_float(row_bcast_i<P>(__float_as_int(v.y))));
}
template <int P> __device__ __forceinline__ double2 row_bcast(double2 v) {
    return make_double2(__hiloint2double(row_bcast_i<P>(__double2hiint(v.x)), row_bcast_i<P>(__double2loint(v.x))),
                        __hiloint2double(row_bcast_i<P>(__double2hiint(v.y)), row_bcast_i<P>(__double2loint(v.y))));
}

// One pivot of gj16_wave (below).
template <typename T, int P>
__device__ __forceinline__ void gj16_pivot(typename CT<T>::c (&a)[4], float thr, bool& small, int r, int g) {
    using C = typename CT<T>::c;
    constexpr int GP = P >> 2, EP = P & 3;
    const C f0 = lane_read(a[EP], r + 16 * GP);            // a[r][p], from another row of lanes
    C pr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) pr[e] = row_bcast<P>(a[e]);   // a[p][4g + e], lane p of this row of lanes
    const C piv = lane_bcast(a[EP], P + 16 * GP);          // a[p][p]
    if (!((float)(piv.x * piv.x + piv.y * piv.y) >= thr)) small = true;
    const C dv = crcp(piv);
    C f = f0;
    if (r == P) f.x -= (T)1;
    const C fs = cmul(f, dv);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const C up = mk<C>(fma(-fs.x, pr[e].x, fma(fs.y, pr[e].y, a[e].x)),
                           fma(-fs.x, pr[e].y, fma(-fs.y, pr[e].x, a[e].y)));
        if (e == EP) a[e] = HELM_CSEL(g == GP, mk<C>((r == P ? (T)1 : (T)0) - fs.x, -fs.y), up);
        else a[e] = up;
    }
}

// Unpivoted Gauss-Jordan of a 16 x 16 tile held by one wavefront (layout
// above), in a uniform form with no special case for the pivot row: for
// pivot p, with f = (column p) - e_p and d = 1 / a_pp, every entry off
// column p takes a_ij -= (f_i d) a_pj, and column p becomes e_p - f d, which
// leaves the inverse in place.  Every lane reads the old pivot row at its columns and
// its row's entry of column p from the lanes that hold them (the row by a
// DPP broadcast within each row of 16 lanes, the column entry by a
// cross-lane read).  Sets small if |a_pp|^2 < thr for some pivot.
template <typename T>
__device__ __forceinline__ void gj16_wave(typename CT<T>::c (&a)[4], float thr, bool& small) {
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
    gj16_pivot<T, 0>(a, thr, small, r, g);
    gj16_pivot<T, 1>(a, thr, small, r, g);
    gj16_pivot<T, 2>(a, thr, small, r, g);
    gj16_pivot<T, 3>(a, thr, small, r, g);
    gj16_pivot<T, 4>(a, thr, small, r, g);
    gj16_pivot<T, 5>(a, thr, small, r, g);
    gj16_pivot<T, 6>(a, thr, small, r, g);
    gj16_pivot<T, 7>(a, thr, small, r, g);
    gj16_pivot<T, 8>(a, thr, small, r, g);
    gj16_pivot<T, 9>(a, thr, small, r, g);
    gj16_pivot<T, 10>(a, thr, small, r, g);
    gj16_pivot<T, 11>(a, thr, small, r, g);
    gj16_pivot<T, 12>(a, thr, small, r, g);
    gj16_pivot<T, 13>(a, thr, small, r, g);
    gj16_pivot<T, 14>(a, thr, small, r, g);
    gj16_pivot<T, 15>(a, thr, small, r, g);
}

// D = Cadd + sign * A B for 16 x 16 complex blocks in LDS (row stride 33),
// by one wavefront on the matrix cores; Cadd may be null.  D may alias Cadd
// (each lane reads its own entries of Cadd before writing them) but not A
// or B.
template <typename T>
__device__ __forceinline__ void mm16(const typename CT<T>::c* A, const typename CT<T>::c* B,
                                     const typename CT<T>::c* Cadd, typename CT<T>::c* D, T sign) {
    using C = typename CT<T>::c;
    using V = typename CT<T>::v4;
    const int l = threadIdx.x & 63, lr = l & 15, lg = l >> 4;
    V re, im;
#pragma unroll
    for (int e = 0; e < 4; ++e) { re[e] = 0; im[e] = 0; }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const C x = A[lr * 33 + 4 * q + lg], y = B[(4 * q + lg) * 33 + lr];
        cmfma<T, V>(re, im, x.x, x.y, y.x, y.y);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = acc_row<T>(lg, e);
        C v = mk<C>(sign * re[e], sign * im[e]);
        if (Cadd) v = cadd(Cadd[row * 33 + lr], v);
        D[row * 33 + lr] = v;
    }
}

// The unpivoted inverse of the kb x kb tile in a[] (256-thread layout of the
// pivoted path: thread t holds row t / 8, columns 4 (t % 8) .. +3), kb = 16
// or 32, left in L[0..kb)[0..kb) (row stride 33; L2 two such buffers).
// Returns whether a pivot was below tau2 * max|tile|^2.
// The second half: the tile already in L2 (rows 0 .. kb-1, stride 33),
// each wavefront's largest |a_ij|^2 in sh.amax and sh.small cleared, all
// visible to the workgroup.
template <typename T>
__device__ __forceinline__ bool inv_blocked_core(int kb, typename CT<T>::c* L2, RowScratch<T>& sh, float tau2);

template <typename T>
__device__ __forceinline__ bool inv_blocked(typename CT<T>::c (&a)[4], int kb, typename CT<T>::c* L2,
                                            RowScratch<T>& sh, float tau2) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int r = t >> 3, cg = t & 7;
    const bool act = (r < kb) && (4 * cg < kb);
    {
        float m2 = 0.0f;
        if (act) {
#pragma unroll
            for (int e = 0; e < 4; ++e) m2 = fmaxf(m2, (float)(a[e].x * a[e].x + a[e].y * a[e].y));
        }
        const uint32_t wm = wave_max_u32(__float_as_uint(m2));
        if (l == 0) sh.amax[w] = __uint_as_float(wm);
        if (t == 0) sh.small = 0;
        if (act) {
#pragma unroll
            for (int e = 0; e < 4; ++e) L2[r * 33 + 4 * cg + e] = a[e];
        }
    }
    __syncthreads();
    return inv_blocked_core<T>(kb, L2, sh, tau2);
}

template <typename T>
__device__ __forceinline__ bool inv_blocked_core(int kb, typename CT<T>::c* L2, RowScratch<T>& sh, float tau2) {
    using C = typename CT<T>::c;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    C* L = L2;               // the tile, then its inverse
    C* Lb = L2 + 32 * 33;    // X (rows 0..15) and Y (rows 16..31)
    const float thr = tau2 * fmaxf(fmaxf(sh.amax[0], sh.amax[1]), fmaxf(sh.amax[2], sh.amax[3]));
    const int lr = l & 15, lg = l >> 4;
    bool small = false;
    // A^-1 in place (wave 0)
    if (w == 0) {
        C q[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) q[e] = L[lr * 33 + 4 * lg + e];
        gj16_wave<T>(q, thr, small);
#pragma unroll
        for (int e = 0; e < 4; ++e) L[lr * 33 + 4 * lg + e] = q[e];
    }
    if (kb == 32) {
        __syncthreads();
        if (w == 0) mm16<T>(L, L + 16, nullptr, Lb, (T)1);                          // X = A^-1 B
        else if (w == 1) mm16<T>(L + 16 * 33, L, nullptr, Lb + 16 * 33, (T)1);       // Y = C A^-1
        __syncthreads();
        if (w == 0) mm16<T>(Lb + 16 * 33, L + 16, L + 16 * 33 + 16, L + 16 * 33 + 16, (T)-1);   // S = D - Y B
        __syncthreads();
        if (w == 0) {
            C q[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) q[e] = L[(16 + lr) * 33 + 16 + 4 * lg + e];
            gj16_wave<T>(q, thr, small);
#pragma unroll
            for (int e = 0; e < 4; ++e) L[(16 + lr) * 33 + 16 + 4 * lg + e] = q[e];
        }
        __syncthreads();
        if (w == 0) mm16<T>(Lb, L + 16 * 33 + 16, nullptr, L + 16, (T)-1);              // T12 = -X S^-1
        else if (w == 1) mm16<T>(L + 16 * 33 + 16, Lb + 16 * 33, nullptr, L + 16 * 33, (T)-1);   // T21 = -S^-1 Y
        __syncthreads();
        if (w == 0) mm16<T>(Lb, L + 16 * 33, L, L, (T)-1);                              // T11 = A^-1 - X T21
    }
    if (small) sh.small = 1;
    __syncthreads();
    return sh.small != 0;
}

// Device-coherent store of one complex64 value: a relaxed agent-scope atomic
// store, which writes through the XCD's L2 to memory.
__device__ __forceinline__ void cst(float2* p, float2 v) {
    const unsigned long long w = (unsigned long long)__float_as_uint(v.x) |
                                 ((unsigned long long)__float_as_uint(v.y) << 32);
    __hip_atomic_store((HELM_GLOBAL unsigned long long*)p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Store of an updated panel element.  Complex64: a device-coherent store
// (written through to memory, no dirty line left in the XCD's L2); with
// every step rewriting the whole block, lines left dirty at the end of a
// launch delay the start of the next launch's workgroups (measured: the
// last workgroups entered ~4 us after the first, ~2 us with these stores).
// Complex128: a non-temporal store (two coherent 8-byte halves cost more
// than they save).
__device__ __forceinline__ void yst(float2* p, float2 v) { cst(p, v); }
__device__ __forceinline__ void yst(double2* p, double2 v) {
    gv2d w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, (HELM_GLOBAL gv2d*)p);
}

// Pivot tolerance of the unpivoted path: |a_pp|^2 >= TAU2 * max|a|^2.
constexpr float TAU2 = 1e-4f;

// The unpivoted inverse in L2 (stride 33) to Tt, transposed, row stride KB.
// Tt is device memory (the factor's tile slots) or LDS (the standalone
// tile-inverse kernel), so it is written through a generic pointer.
template <typename T>
__device__ __forceinline__ void store_inverse(int kb, const typename CT<T>::c* L2, typename CT<T>::c* Tt) {
    const int t = threadIdx.x, r = t >> 3, cg = t & 7;
    if ((r < kb) && (4 * cg < kb)) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 4 * cg + e;
            Tt[c * KB + r] = L2[r * 33 + c];
        }
    }
}

// Invert the kb x kb tile in a[] and store its inverse transposed
// (Tt[c][k] = T^{-1}[k][c]) with row stride KB.  M is a kb x 33 LDS buffer
// (pivoted path), L2 two 32 x 33 LDS buffers (unpivoted path).  Returns the
// first zero-pivot step (pivoted path) or -1; *small is set when the
// unpivoted path met a pivot below the tolerance.  Tt may be device memory
// or LDS (generic stores).
template <typename T>
__device__ __forceinline__ int invert_and_store(typename CT<T>::c (&a)[4], int kb, int pivot, GJScratch<T>& sh,
                                                typename CT<T>::c (*M)[33], typename CT<T>::c* L2,
                                                typename CT<T>::c* Tt, bool* small) {
    const int t = threadIdx.x, r = t >> 3, cg = t & 7;
    const bool act = (r < kb) && (4 * cg < kb);
    if (!pivot) {
        // diagonal pivots: the blocked form (two 16 x 16 inverses in one
        // wavefront each, the products around them on the matrix cores)
        RowScratch<T>& rs = *(RowScratch<T>*)&sh;
        *small = inv_blocked<T>(a, kb, L2, rs, TAU2);
        store_inverse<T>(kb, L2, Tt);
        return -1;
    }
    *small = false;
    int zero = (kb == 32) ? gj_invert<T, 32>(a, sh) : gj_invert<T, 16>(a, sh);
    if (act) {
#pragma unroll
        for (int e = 0; e < 4; ++e) M[r][4 * cg + e] = a[e];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 4 * cg + e;
            Tt[c * KB + r] = M[sh.rowOf[r]][sh.stepOf[c]];
        }
    }
    return zero;
}

__device__ __forceinline__ void report_zero_pivot(int* status, int block, int row) {
    if (atomicCAS(&status[0], 0, 1) == 0) {
        status[1] = block;
        status[2] = row;
    }
}

// ----------------------------------------------------------------- launches --
// LDS of a step workgroup: update tiles use sW, sV (64 x 33 each); the
// next-tile workgroup four 32 x 33 blocks and the pivoting scratch
template <typename T>
constexpr size_t sm_bytes() {
    using C = typename CT<T>::c;
    constexpr size_t upd = 2 * 64 * 33 * sizeof(C), nxt = 4 * 32 * 33 * sizeof(C) + sizeof(GJScratch<T>);
    return upd > nxt ? upd : nxt;
}

__host__ __device__ int init_blocks(int np) { return (int)(((int64_t)np * np + 255) / 256) + 1; }
__host__ __device__ int step_blocks(int np) {
    const int tx = (np + TILE - 1) / TILE;
    return tx * tx + 1;
}
int factor_init_blocks(int np) { return init_blocks(np); }
int factor_step_blocks(int np) { return step_blocks(np); }

// D = A_{row0} into the first block of each front, and the inverse of its
// first diagonal tile
template <typename T>
__global__ __launch_bounds__(256) void k_factor_init(const ChainTab* __restrict__ tab, int n) {
    using C = typename CT<T>::c;
    __shared__ C M[32][33];
    __shared__ C L2[2 * 32 * 33];
    __shared__ GJScratch<T> sh;
    const int ci = find_chain(tab->c, n, blockIdx.x, [](const ChainInfo& c) { return c.itile0; });
    const ChainInfo d = load_entry(tab->c, ci);
    const int local = blockIdx.x - d.itile0;
    const int np = d.np;
    const int nfill = init_blocks(np) - 1;
    if (local < nfill) {
        const int64_t e = (int64_t)local * 256 + threadIdx.x;
        if (e < (int64_t)np * np) {
            const int r = (int)(e / np), q = (int)(e % np);
            const double2 v = block_entry(d.cf, d.row0, r, q);
            ((C*)d.G)[(size_t)d.row0 * np * np + e] = mk<C>(v.x, v.y);
        }
        return;
    }
    const int kb = min(KB, np);
    const int t = threadIdx.x, r = t >> 3, cg = t & 7;
    C a[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = 4 * cg + e;
        const double2 v = (r < kb && c < kb) ? block_entry(d.cf, d.row0, r, c) : make_double2(0.0, 0.0);
        a[e] = mk<C>(v.x, v.y);
    }
    bool small;
    const int zero = invert_and_store<T>(a, kb, d.pivot, sh, M, L2, (C*)d.Tb, &small);
    if (zero >= 0 && t == 0) report_zero_pivot(d.status, d.row0, zero);
    if (small && t == 0) d.status[3] = 1;
}

// Source of A for the block after local block jl of a front: the merge
// block for the top front's last block, else null (assemble from m).
template <typename C>
__device__ __forceinline__ const C* next_a_source(const ChainInfo& d, int jl) {
    return (d.Ain && jl + 1 == d.nblk - 1) ? (const C*)d.Ain : nullptr;
}

// Entry (r, c) of the next block's first diagonal tile, A_{j+1} - E G_j E,
// from the entry g of G_j (the Schur complement on a block's last panel).
template <typename C>
__device__ __forceinline__ C next_schur(const ChainInfo& d, const C* Asrc, int jn, int r, int c, C g) {
    double2 a1;
    if (Asrc) {
        const C v = gld(Asrc + (size_t)r * d.np + c);
        a1 = make_double2(v.x, v.y);
    } else {
        a1 = block_entry(d.cf, jn, r, c);
    }
    const double s = row_coupling(d.cf, r) * row_coupling(d.cf, c);
    return mk<C>(a1.x - s * (double)g.x, a1.y - s * (double)g.y);
}

// workgroup that prepares the next step's inverted diagonal tile
template <typename T>
__device__ __forceinline__ void next_tile(const ChainInfo& d, const PanelStep& ps, const typename CT<T>::c* X,
                          const typename CT<T>::c* Tcur, typename CT<T>::c* Tnext, char* smem) {
    using C = typename CT<T>::c;
    const int np = d.np, kb = ps.kb, k0 = ps.k0;
    const int row = d.row0 + d.dir * ps.j;
    int jn, kn0, kbn;
    const C* Asrc = nullptr;
    if (!ps.last_panel) {
        jn = row;
        kn0 = k0 + kb;
    } else {
        if (ps.j + 1 >= d.nblk) return;
        jn = row + d.dir;
        kn0 = 0;
        Asrc = next_a_source<C>(d, ps.j);
    }
    kbn = min(KB, np - kn0);
    C (*sXa)[33] = (C(*)[33])smem;                      // X_{K'K}    kbn x kb
    C (*sT)[33] = (C(*)[33])(smem + 1 * 32 * 33 * sizeof(C));   // T   kb x kb
    C (*sXb)[33] = (C(*)[33])(smem + 2 * 32 * 33 * sizeof(C));  // X_{KK'}    kb x kbn
    C (*sP)[33] = (C(*)[33])(smem + 3 * 32 * 33 * sizeof(C));   // X_{K'K} T  kbn x kb
    GJScratch<T>& sh = *(GJScratch<T>*)(smem + 4 * 32 * 33 * sizeof(C));
    const int t = threadIdx.x, r = t >> 3, cg = t & 7;
    const bool single = ps.last_panel && d.npan == 1;   // next tile is Y = T itself
    const int w = t >> 6, l = t & 63, lr = l & 15, lg = l >> 4;
    const int wr = w >> 1, wc = w & 1;   // this wave's 16 x 16 output tile of the products
    // every global load is issued up front at a clamped (in-range) address;
    // entries outside the kb x kbn tiles are zeroed when they are placed.
    // T arrives transposed (Tt[c][k]): read it in order, place it as sT[k][c]
    C tl[4], xa[4], xb[4], xz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = t + 256 * i;
        const int hi = idx >> 5, lo = idx & 31;
        tl[i] = gld(Tcur + idx);
        xa[i] = gld(X + (size_t)(kn0 + min(hi, kbn - 1)) * np + k0 + min(lo, kb - 1));
        xb[i] = gld(X + (size_t)(k0 + min(hi, kb - 1)) * np + kn0 + min(lo, kbn - 1));
    }
    // X_{K'K'} in the accumulator layout of this wave's tile
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int rr = 16 * wr + acc_row<T>(lg, e), cc = 16 * wc + lr;
        xz[e] = gld(X + (size_t)(kn0 + min(rr, kbn - 1)) * np + kn0 + min(cc, kbn - 1));
    }
    __builtin_amdgcn_sched_barrier(0);   // keep every load ahead of the first wait
    const C cz = mk<C>(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = t + 256 * i;
        const int hi = idx >> 5, lo = idx & 31;
        sT[lo][hi] = HELM_CSEL(hi < kb && lo < kb, tl[i], cz);
        sXa[hi][lo] = HELM_CSEL(!single && hi < kbn && lo < kb, xa[i], cz);
        sXb[hi][lo] = HELM_CSEL(!single && hi < kb && lo < kbn, xb[i], cz);
    }
    using V = typename CT<T>::v4;
    V zr, zi;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int rr = 16 * wr + acc_row<T>(lg, e), cc = 16 * wc + lr;
        const C v = HELM_CSEL(!single && rr < kbn && cc < kbn, xz[e], cz);
        zr[e] = v.x;
        zi[e] = v.y;
    }
    C a[4];
    const bool act = (r < kbn) && (4 * cg < kbn);
    __syncthreads();
    if (single) {
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = HELM_CSEL(act, sT[r][4 * cg + e], mk<C>(0.0, 0.0));
    } else {
        // P = X_{K'K} T on the matrix cores (zero padding beyond kb, kbn), in
        // three real products per complex one like the update tiles' W
        V pr, pim;
        {
            V p1, p2, p3;
#pragma unroll
            for (int e = 0; e < 4; ++e) { p1[e] = 0; p2[e] = 0; p3[e] = 0; }
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                const C x = sXa[16 * wr + lr][4 * s8 + lg], y = sT[4 * s8 + lg][16 * wc + lr];
                cacc<true, T, V>(p1, p2, p3, x.x, x.y, y.x, y.y);
            }
            cacc_final<true, V>(p1, p2, p3, pr, pim);
        }
        // -P into sP (accumulator layout -> row-major)
#pragma unroll
        for (int e = 0; e < 4; ++e) sP[16 * wr + acc_row<T>(lg, e)][16 * wc + lr] = mk<C>(-pr[e], -pim[e]);
        __syncthreads();
        // Z = X_{K'K'} - P X_{KK'}
#pragma unroll
        for (int s8 = 0; s8 < 8; ++s8) {
            const C x = sP[16 * wr + lr][4 * s8 + lg], y = sXb[4 * s8 + lg][16 * wc + lr];
            cmfma<T, V>(zr, zi, x.x, x.y, y.x, y.y);
        }
        if (!d.pivot) {
            // unpivoted: each wave puts its block of the tile (after the
            // Schur complement of the next block on a last panel) straight
            // into the inversion buffer and reports its largest |a_ij|^2
            C* L2 = &sT[0][0];   // T and X_{KK'} are no longer read there
            RowScratch<T>& rs = *(RowScratch<T>*)&sh;
            float m2 = 0.0f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rr = 16 * wr + acc_row<T>(lg, e), cc = 16 * wc + lr;
                C v = mk<C>(0.0, 0.0);
                if (rr < kbn && cc < kbn) {
                    v = mk<C>(zr[e], zi[e]);
                    if (ps.last_panel) v = next_schur<C>(d, Asrc, jn, rr, cc, v);
                    m2 = fmaxf(m2, (float)(v.x * v.x + v.y * v.y));
                }
                L2[rr * 33 + cc] = v;
            }
            const uint32_t wm = wave_max_u32(__float_as_uint(m2));
            if (l == 0) rs.amax[w] = __uint_as_float(wm);
            if (t == 0) rs.small = 0;
            __syncthreads();
            const bool small = inv_blocked_core<T>(kbn, L2, rs, TAU2);
            store_inverse<T>(kbn, L2, Tnext);
            if (small && t == 0) d.status[3] = 1;
            return;
        }
        // to the Gauss-Jordan layout through sXa (no longer read)
#pragma unroll
        for (int e = 0; e < 4; ++e) sXa[16 * wr + acc_row<T>(lg, e)][16 * wc + lr] = mk<C>(zr[e], zi[e]);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = HELM_CSEL(act, sXa[r][4 * cg + e], mk<C>(0.0, 0.0));
    }
    if (ps.last_panel && act) {
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = next_schur<C>(d, Asrc, jn, r, 4 * cg + e, a[e]);
    }
    __syncthreads();   // sXa is reused as the inversion buffer
    bool small;
    const int zero = invert_and_store<T>(a, kbn, d.pivot, sh, sXa, &sT[0][0], Tnext, &small);
    if (zero >= 0 && t == 0) report_zero_pivot(d.status, jn, kn0 + zero);
    if (small && t == 0) d.status[3] = 1;
}

// Accumulators of the update tile's product seeded with its tile of X'
// (identity on the panel columns K, zero outside the block)
template <bool GAUSS, typename T, typename V, typename C>
__device__ __forceinline__ void seed_y(V (&a1)[2][2], V (&a2)[2][2], V (&a3)[2][2], const C (&xt)[2][2][4],
                                       const int (&R)[2], const int (&Cc)[2], const bool (&vr)[2], const bool (&vc)[2],
                                       int k0, int kb, int lr, int lg) {
    const C zero = mk<C>(0.0, 0.0);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int col = Cc[bj] + lr;
            const bool inK = col >= k0 && col < k0 + kb;
            V sre, sim;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = R[bi] + acc_row<T>(lg, e);
                C v = HELM_CSEL(inK, mk<C>(row == col ? 1.0 : 0.0, 0.0), xt[bi][bj][e]);
                // complex128 selects part by part; complex64 keeps the branch
                if constexpr (sizeof(T) == 8) v = HELM_CSEL(vr[bi] && vc[bj], v, zero);
                else if (!(vr[bi] && vc[bj])) v = zero;
                sre[e] = v.x;
                sim[e] = v.y;
            }
            cacc_seed<GAUSS, V>(a1[bi][bj], a2[bi][bj], a3[bi][bj], sre, sim);
        }
}

// update of one 64 x 64 tile of Y
template <typename T>
__device__ __forceinline__ void update_tile(const ChainInfo& d, const PanelStep& ps, int ti, const typename CT<T>::c* X,
                            typename CT<T>::c* Y, const typename CT<T>::c* Tcur, char* smem) {
    using C = typename CT<T>::c;
    using V = typename CT<T>::v4;
    // three real products per complex one (Gauss) for the Y product in
    // complex128 only: in complex64 its larger rounding of the imaginary
    // parts costs a refinement step.  The W product takes three in both
    // precisions (the complex64 refinement count is unchanged).
    constexpr bool GAUSS = sizeof(T) == 8;
    const int np = d.np, kb = ps.kb, k0 = ps.k0;
    const int tiles_x = (np + TILE - 1) / TILE;
    const int I0 = (ti / tiles_x) * TILE, J0 = (ti % tiles_x) * TILE;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int lr = l & 15, lg = l >> 4;
    const int wr = w >> 1, wc = w & 1;
    C (*sW)[33] = (C(*)[33])smem;                      // W rows I0..I0+63, k < kb
    C (*sV)[33] = (C(*)[33])(smem + 64 * 33 * sizeof(C));  // V^T: sV[c][k], c = J0..J0+63

    int R[2], Cc[2];
    bool vr[2], vc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        R[q] = I0 + 32 * wr + 16 * q;
        Cc[q] = J0 + 32 * wc + 16 * q;
        vr[q] = R[q] < np;
        vc[q] = Cc[q] < np;
    }
    // 1. global loads, all issued up front: X_{I,K} (rows of this tile, panel
    //    columns) and T for the W product, V_J = X_{K,J} for the update (kept
    //    in registers until W is done), and this tile of X'
    C (*sT)[33] = sV;   // T shares the V buffer until W is formed
    // every load is issued at a clamped (in-range) address; out-of-range and
    // identity entries are substituted afterwards
    C xik[8], tv[4], vv[8], xt[2][2][4];
    {
        const int rr = t >> 2, c8 = 8 * (t & 3), row = min(I0 + rr, np - 1);
#pragma unroll
        for (int q = 0; q < 8; ++q) xik[q] = gld(X + (size_t)row * np + k0 + min(c8 + q, kb - 1));
#pragma unroll
        for (int q = 0; q < 4; ++q) tv[q] = gld(Tcur + t + 256 * q);   // Tt[c][k], idx = 32 c + k
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = t + 256 * q, k = i >> 6, cc = i & 63;
            vv[q] = gld(X + (size_t)(k0 + min(k, kb - 1)) * np + min(J0 + cc, np - 1));
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    xt[bi][bj][e] = gld(X + (size_t)min(R[bi] + acc_row<T>(lg, e), np - 1) * np +
                                        min(Cc[bj] + lr, np - 1));
    }
    __builtin_amdgcn_sched_barrier(0);   // keep every load ahead of the first wait
    const C zero = mk<C>(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int i = t + 256 * q, k = i >> 6, col = J0 + (i & 63);
        if constexpr (sizeof(T) == 8) {   // part by part, as above
            vv[q] = HELM_CSEL(col >= k0 && col < k0 + kb, mk<C>(k == col - k0 ? 1.0 : 0.0, 0.0), vv[q]);
            vv[q] = HELM_CSEL(k < kb && col < np, vv[q], zero);
        } else {
            if (!(k < kb && col < np)) vv[q] = zero;
            else if (col >= k0 && col < k0 + kb) vv[q] = mk<C>(k == col - k0 ? 1.0 : 0.0, 0.0);
        }
    }
    // Y = X' + W V, accumulated from X'.  complex128 seeds its three
    // accumulators after the W product: across it the tile of X' (64
    // registers) is live instead of them (96), which keeps the kernel from
    // spilling
    V a1[2][2], a2[2][2], a3[2][2];
    if constexpr (!GAUSS) seed_y<GAUSS, T>(a1, a2, a3, xt, R, Cc, vr, vc, k0, kb, lr, lg);
    // 2. X_{I,K} and T into LDS
    {
        const int rr = t >> 2, c8 = 8 * (t & 3);
        const bool rok = I0 + rr < np;
#pragma unroll
        for (int q = 0; q < 8; ++q) sW[rr][c8 + q] = HELM_CSEL(rok && c8 + q < kb, xik[q], zero);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = t + 256 * q, c = i >> 5, k = i & 31;
            sT[k][c] = HELM_CSEL(k < kb && c < kb, tv[q], mk<C>(0.0, 0.0));
        }
    }
    __syncthreads();
    // 3. W_I = -X_{I,K} T (matrix cores; wave w makes rows I0+16w .. +15), T - I on rows of K
    {
        V wre[2], wim[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            V q1, q2, q3;
#pragma unroll
            for (int e = 0; e < 4; ++e) { q1[e] = 0; q2[e] = 0; q3[e] = 0; }
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                const int k = 4 * s8 + lg;
                const C av = sW[16 * w + lr][k], bv = sT[k][cb * 16 + lr];
                cacc<true, T, V>(q1, q2, q3, av.x, av.y, bv.x, bv.y);
            }
            cacc_final<true, V>(q1, q2, q3, wre[cb], wim[cb]);
        }
        C tk[2][4];   // rows of K: T - I, read before the buffers are rewritten
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = I0 + 16 * w + acc_row<T>(lg, e), c = cb * 16 + lr;
                tk[cb][e] = HELM_CSEL(row >= k0 && row < k0 + kb, sT[row - k0][c], mk<C>(0.0, 0.0));
            }
        __syncthreads();   // every wave has read X_{I,K} and T
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rl = 16 * w + acc_row<T>(lg, e), row = I0 + rl, c = cb * 16 + lr;
                C v;
                if (row >= k0 && row < k0 + kb) {
                    v = tk[cb][e];
                    if (row - k0 == c) v.x -= (T)1;
                } else {
                    v = mk<C>(-wre[cb][e], -wim[cb][e]);
                }
                sW[rl][c] = v;
            }
        }
        // V_J into LDS, transposed (V_KK = I)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = t + 256 * q, k = i >> 6, cc = i & 63;
            sV[cc][k] = vv[q];
        }
    }
    if constexpr (GAUSS) seed_y<GAUSS, T>(a1, a2, a3, xt, R, Cc, vr, vc, k0, kb, lr, lg);
    __syncthreads();
    // 4. Y_IJ = X'_IJ + W_I V_J
    for (int kk = 0; kk < kb; kk += 16) {
        C av[2][4], bv[2][4];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                av[q][s] = sW[32 * wr + 16 * q + lr][kk + 4 * lg + s];
                bv[q][s] = sV[32 * wc + 16 * q + lr][kk + 4 * lg + s];
            }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    if (vr[bi] && vc[bj])
                        cacc<GAUSS, T, V>(a1[bi][bj], a2[bi][bj], a3[bi][bj], av[bi][s].x, av[bi][s].y, bv[bj][s].x,
                                          bv[bj][s].y);
    }
    // 5. store; after the last panel also D_next = A_next - E Y E, into the
    //    front's next block, or into the merge block after a bottom front's
    //    last block
    const int row_b = d.row0 + d.dir * ps.j, rn = row_b + d.dir;
    C* An = nullptr;
    const C* Asrc = nullptr;
    if (ps.last_panel) {
        if (ps.j + 1 < d.nblk) {
            An = (C*)d.G + (size_t)rn * np * np;
            Asrc = next_a_source<C>(d, ps.j);
        } else if (d.Aout) {
            An = (C*)d.Aout;
        }
    }
    const bool schur = An != nullptr;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            if (!(vr[bi] && vc[bj])) continue;
            const int col = Cc[bj] + lr;
            V gre, gim;
            cacc_final<GAUSS, V>(a1[bi][bj], a2[bi][bj], a3[bi][bj], gre, gim);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = R[bi] + acc_row<T>(lg, e);
                const C g = mk<C>(gre[e], gim[e]);
                // the finished inverse goes to the sweeps' operand layout
                yst(Y + (ps.last_panel ? (sizeof(T) == 4 ? a_tiled4(row, col, np) : a_tiled(row, col, np))
                                       : (size_t)row * np + col),
                    g);
                if (schur) {
                    double2 a1;
                    if (Asrc) {
                        const C v = gld(Asrc + (size_t)row * np + col);
                        a1 = make_double2(v.x, v.y);
                    } else {
                        a1 = block_entry(d.cf, rn, row, col);
                    }
                    const double s = row_coupling(d.cf, row) * row_coupling(d.cf, col);
                    yst(An + (size_t)row * np + col, mk<C>(a1.x - s * (double)g.x, a1.y - s * (double)g.y));
                }
            }
        }
}

// Workgroups 0 .. n-1 of a step launch prepare the next diagonal tile of
// chains 0 .. n-1 (the critical path of the step, so they are dispatched
// first); the rest update the 64 x 64 tiles, chain by chain (ftile0).
// uni > 0: every chain has uni - 1 update workgroups, laid out by XCD
// (xcd_tile); otherwise in launch order.
// Update tile served by workgroup b (>= n) when consecutive tiles (front by
// front, tile row by tile row) are kept on one XCD: workgroup b runs on XCD
// b % 8, so XCD x takes the contiguous range of tiles after those of XCDs
// 0 .. x-1, and the panel rows, columns and T of a front are fetched into
// one or two L2s instead of all eight.  total = n + update tiles.
__device__ __forceinline__ int xcd_tile(int b, int n, int total) {
    const int x = b & 7, k = b >> 3;
    int start = 0, leads_x = 0;
#pragma unroll
    for (int y = 0; y < 8; ++y) {
        const int wgs = total > y ? (total - 1 - y) / 8 + 1 : 0;
        const int leads = n > y ? (n - 1 - y) / 8 + 1 : 0;
        if (y < x) start += wgs - leads;
        if (y == x) leads_x = leads;
    }
    return start + k - leads_x;
}

template <typename T>
__global__ __launch_bounds__(256, 2) void k_factor_step(int n, int tstep, int uni, const ChainTab* __restrict__ tab) {
    using C = typename CT<T>::c;
    __shared__ __attribute__((aligned(16))) char smem[sm_bytes<T>()];
    const int b = blockIdx.x;
    const bool nxt = b < n;
    const int u = (!nxt && uni > 0) ? xcd_tile(b, n, n * uni) : b - n;
    const int ci = nxt ? b
                       : uni > 0 ? (int)((unsigned)u / (unsigned)(uni - 1))
                                 : find_chain(tab->c, n, u, [](const ChainInfo& c) { return c.ftile0; });
    const ChainInfo d = load_entry(tab->c, ci);
    if (tstep >= d.T) return;
    const PanelStep ps = panel_step(d, tstep);
    const int np = d.np;
    const size_t n2 = (size_t)np * np;
    C* G = (C*)d.G;
    const int row = d.row0 + d.dir * ps.j;
    const C* X = ps.p == 0 ? G + (size_t)row * n2 : (const C*)((ps.p - 1) & 1 ? d.P1 : d.P0);
    C* Y = ps.last_panel ? G + (size_t)row * n2 : (C*)(ps.p & 1 ? d.P1 : d.P0);
    const C* Tcur = (const C*)d.Tb + (size_t)(tstep & 1) * KB * KB;
    C* Tnext = (C*)d.Tb + (size_t)((tstep + 1) & 1) * KB * KB;
    if (nxt) {
        next_tile<T>(d, ps, X, Tcur, Tnext, smem);
    } else {
        update_tile<T>(d, ps, u - d.ftile0, X, Y, Tcur, smem);
    }
}

// standalone tile inverses (the building block above, for tests)
__global__ __launch_bounds__(256) void k_tile_inverse(int kb, int pivot, const double2* A, double2* Tout, int* status) {
    __shared__ double2 M[32][33];
    __shared__ double2 L2[2 * 32 * 33];
    __shared__ GJScratch<double> sh;
    __shared__ double2 Tt[KB * KB];
    const int t = threadIdx.x, r = t >> 3, cg = t & 7;
    const double2* Am = A + (size_t)blockIdx.x * kb * kb;
    double2 a[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = 4 * cg + e;
        a[e] = (r < kb && c < kb) ? Am[r * kb + c] : make_double2(0.0, 0.0);
    }
    bool small;
    const int zero = invert_and_store<double>(a, kb, pivot, sh, M, L2, Tt, &small);
    __syncthreads();
    for (int i = t; i < kb * kb; i += 256) {
        const int rr = i / kb, c = i % kb;
        Tout[(size_t)blockIdx.x * kb * kb + i] = Tt[c * KB + rr];
    }
    if (t == 0 && zero >= 0) status[blockIdx.x] = 1 + zero;
    if (t == 0 && small) status[blockIdx.x] = -1;
}

void launch_factor_init(const ChainTab* dtab, int n, int total, bool fp32, hipStream_t st) {
    if (fp32) hipLaunchKernelGGL(k_factor_init<float>, dim3(total), dim3(256), 0, st, dtab, n);
    else hipLaunchKernelGGL(k_factor_init<double>, dim3(total), dim3(256), 0, st, dtab, n);
}
int factor_uniform(const ChainTab& tab, int n) {
    int uni = step_blocks(tab.c[0].np);
    for (int q = 0; q < n; ++q)
        if (tab.c[q].ftile0 != q * (uni - 1) || step_blocks(tab.c[q].np) != uni) uni = 0;
    return uni;
}
void launch_factor_step(const ChainTab* dtab, int n, int t, int uni, int total, bool fp32, hipStream_t st) {
    if (fp32) hipLaunchKernelGGL(k_factor_step<float>, dim3(total), dim3(256), 0, st, n, t, uni, dtab);
    else hipLaunchKernelGGL(k_factor_step<double>, dim3(total), dim3(256), 0, st, n, t, uni, dtab);
}
void launch_tile_inverse(int count, int kb, int pivot, const double* A, double* T, int* status, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_inverse, dim3(count), dim3(256), 0, st, kb, pivot, (const double2*)A, (double2*)T,
                       status);
}

}  // namespace helm
