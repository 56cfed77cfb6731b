// Device-side helpers shared by the HIP kernels of libhelm: complex
// arithmetic, the matrix-core wrappers, and on-the-fly assembly of the
// five-point operator A(m, w) of App. A.1 (arXiv 2301.10762).
#pragma once
#include "helm_internal.h"

namespace helm {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct CT;
template <> struct CT<double> { using c = double2; using v4 = v4d; };
template <> struct CT<float> { using c = float2; using v4 = v4f; };

template <typename C> __device__ __forceinline__ C mk(double re, double im) { C r; r.x = re; r.y = im; return r; }
// p ? a : b for complex values.  A select of whole double2 values can be
// lowered to a copy of both into a stack array and a load from the chosen
// address (which also waits for every load in flight), so complex128 values
// are chosen part by part.  float2 values keep the plain conditional, which
// the compiler handles well (the size test is a constant: only one arm is
// emitted).
template <typename C> __device__ __forceinline__ C csel_parts(bool p, C a, C b) {
    C r;
    r.x = p ? a.x : b.x;
    r.y = p ? a.y : b.y;
    return r;
}
#define HELM_CSEL(p, a, b) (sizeof((a).x) == 8 ? csel_parts((p), (a), (b)) : ((p) ? (a) : (b)))

// Loads and stores through pointers read from the device-side tables.  The
// compiler cannot tell that such generic pointers address global memory and
// would emit flat instructions, whose completion is counted together with
// LDS and scalar traffic (so every wait drains everything); these give
// global_* instructions.
#define HELM_GLOBAL __attribute__((address_space(1)))
typedef double gv2d __attribute__((ext_vector_type(2)));
typedef float gv2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 gld(const double2* p) {
    const gv2d v = *(const HELM_GLOBAL gv2d*)p;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 gld(const float2* p) {
    const gv2f v = *(const HELM_GLOBAL gv2f*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gst(double2* p, double2 v) {
    gv2d w;
    w.x = v.x;
    w.y = v.y;
    *(HELM_GLOBAL gv2d*)p = w;
}
__device__ __forceinline__ void gst(float2* p, float2 v) {
    gv2f w;
    w.x = v.x;
    w.y = v.y;
    *(HELM_GLOBAL gv2f*)p = w;
}
template <typename C> __device__ __forceinline__ C cmul(C a, C b) { return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, double s) { return mk<C>(a.x * s, a.y * s); }
template <typename C> __device__ __forceinline__ C cconj(C a) { return mk<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cinv(C a) {
    // 1/a with the larger component factored out (Smith's scaling)
    if (fabs((double)a.x) >= fabs((double)a.y)) {
        double r = (double)a.y / (double)a.x, den = (double)a.x + (double)a.y * r;
        return mk<C>(1.0 / den, -r / den);
    } else {
        double r = (double)a.x / (double)a.y, den = (double)a.x * r + (double)a.y;
        return mk<C>(r / den, -1.0 / den);
    }
}

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of the 16x16 result held in accumulator element e by lane group g
// (lanes 16g .. 16g+15 hold columns 0..15): the FP64 instruction interleaves
// the rows (g + 4e), the FP32 one keeps them contiguous (4g + e).
template <typename T> __device__ __forceinline__ int acc_row(int g, int e);
template <> __device__ __forceinline__ int acc_row<double>(int g, int e) { return g + 4 * e; }
template <> __device__ __forceinline__ int acc_row<float>(int g, int e) { return 4 * g + e; }

// (cr + i ci) += (ar + i ai)(br + i bi) for one 16x16x4 block
template <typename T, typename V>
__device__ __forceinline__ void cmfma(V& cr, V& ci, T ar, T ai, T br, T bi) {
    cr = mfma16(ar, br, cr);
    cr = mfma16(-ai, bi, cr);
    ci = mfma16(ar, bi, ci);
    ci = mfma16(ai, br, ci);
}

// The same product in three real products (Gauss): p1 += ar br,
// p2 += ai bi, p3 += (ar + ai)(br + bi); then re = p1 - p2 and
// im = p3 - p1 - p2.  An accumulator starting at c is seeded
// p1 = c.re, p2 = 0, p3 = c.re + c.im.
template <typename T, typename V>
__device__ __forceinline__ void cmfma3(V& p1, V& p2, V& p3, T ar, T ai, T br, T bi) {
    p1 = mfma16(ar, br, p1);
    p2 = mfma16(ai, bi, p2);
    p3 = mfma16(ar + ai, br + bi, p3);
}

// Complex product accumulated either way: with GAUSS, (a1, a2, a3) are the
// three-product accumulators above; otherwise a1 = re, a3 = im (four real
// products) and a2 is unused.
template <bool GAUSS, typename T, typename V>
__device__ __forceinline__ void cacc(V& a1, V& a2, V& a3, T ar, T ai, T br, T bi) {
    if constexpr (GAUSS) cmfma3<T, V>(a1, a2, a3, ar, ai, br, bi);
    else cmfma<T, V>(a1, a3, ar, ai, br, bi);
}
template <bool GAUSS, typename V>
__device__ __forceinline__ void cacc_seed(V& a1, V& a2, V& a3, V re, V im) {
    a1 = re;
    a2 = re - re;
    a3 = GAUSS ? re + im : im;
}
template <bool GAUSS, typename V>
__device__ __forceinline__ void cacc_final(V a1, V a2, V a3, V& re, V& im) {
    if constexpr (GAUSS) {
        im = a3 - a1 - a2;
        re = a1 - a2;
    } else {
        re = a1;
        im = a3;
    }
}

// ---------------------------------------------------------------- assembly --
__device__ __forceinline__ double half_at_ends(int idx, int n) { return (idx == 0 || idx == n - 1) ? 0.5 : 1.0; }
__device__ __forceinline__ double x_coupling(const Coef& c, int j) { return (c.hz / c.hx) * half_at_ends(j, c.nz); }
__device__ __forceinline__ double z_coupling(const Coef& c, int i) { return (c.hx / c.hz) * half_at_ends(i, c.nx); }

// A(m, w) at node (i, j), diagonal entry
__device__ __forceinline__ double2 diag_entry(const Coef& c, int i, int j) {
    double cx = x_coupling(c, j), cz = z_coupling(c, i);
    double s = 0.0;
    if (i > 0) s += cx;
    if (i < c.nx - 1) s += cx;
    if (j > 0) s += cz;
    if (j < c.nz - 1) s += cz;
    double mass = c.hx * c.hz * half_at_ends(i, c.nx) * half_at_ends(j, c.nz);
    double bnd = 0.0;
    if (j == 0 || j == c.nz - 1) bnd += 0.5 * c.hx * ((i > 0 ? 1 : 0) + (i < c.nx - 1 ? 1 : 0));
    if (i == 0 || i == c.nx - 1) bnd += 0.5 * c.hz * ((j > 0 ? 1 : 0) + (j < c.nz - 1 ? 1 : 0));
    double mk_ = *((const HELM_GLOBAL double*)c.m + (size_t)j * c.nx + i);
    return make_double2(s - c.omega * c.omega * mass * mk_, -c.omega * bnd * sqrt(mk_));
}

// entry (r, q) of the padded diagonal block A_j (identity in the padding)
__device__ __forceinline__ double2 block_entry(const Coef& c, int j, int r, int q) {
    if (r >= c.nx || q >= c.nx) return make_double2(r == q ? 1.0 : 0.0, 0.0);
    if (r == q) return diag_entry(c, r, j);
    if (r == q + 1 || q == r + 1) return make_double2(-x_coupling(c, j), 0.0);
    return make_double2(0.0, 0.0);
}

// coupling E_ii between rows j and j+1 (zero in the padding)
__device__ __forceinline__ double row_coupling(const Coef& c, int i) { return i < c.nx ? -z_coupling(c, i) : 0.0; }

// Copy of table entry ci (a kernel argument) with every dword read in one
// round of scalar loads.  Left to itself the compiler fetches each field
// where it is first used, after the early exits of a kernel, which chains
// several round trips to the kernel-argument memory.  The empty asm with each
// dword as an in-out scalar operand makes all of them live here.
template <typename Info>
__device__ __forceinline__ Info load_entry(const Info* tab, int ci) {
    static_assert(sizeof(Info) % 4 == 0, "table entries are whole dwords");
    constexpr int W = (int)(sizeof(Info) / 4);
    uint32_t w[W];
    __builtin_memcpy(w, &tab[ci], sizeof(Info));
#pragma unroll
    for (int i = 0; i < W; ++i) asm volatile("" : "+s"(w[i]));
    Info d;
    __builtin_memcpy(&d, w, sizeof(Info));
    return d;
}

// Chain owning work item `bid`, given each chain's first item.  Tables are
// allocated with MAXB entries (unused ones start at INT_MAX), so the scan has
// no data-dependent loads: all entries are fetched at once.
template <typename Info, typename F>
__device__ __forceinline__ int find_chain(const Info* tab, int n, int bid, F first) {
    int c = 0;
#pragma unroll
    for (int q = 1; q < MAXB; ++q) c = (bid >= first(tab[q])) ? q : c;
    return c;
}

// the panel step a chain performs at global step t: block j, panel p
// (columns k0 .. k0+kb-1 of the block)
struct PanelStep {
    int j, p, k0, kb, last_panel;
};
__device__ __forceinline__ PanelStep panel_step(const ChainInfo& c, int t) {
    PanelStep s;
    s.j = t / c.npan;
    s.p = t - s.j * c.npan;
    s.k0 = s.p * KB;
    s.kb = min(KB, c.np - s.k0);
    s.last_panel = s.p == c.npan - 1;
    return s;
}

}  // namespace helm
