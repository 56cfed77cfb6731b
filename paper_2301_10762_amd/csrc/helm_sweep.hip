// Block sweeps of libhelm (gfx950): multi-right-hand-side forward and back
// substitution with the stored Schur-complement inverses G_j,
//     forward   w_j = G_j y_j,          y_{j+dir} = b_{j+dir} - E w_j,
//     backward  x_j = w_j - G_j z_j,    z_{j-dir} = E x_j,
// run from both ends of the grid at once (the two fronts of the twisted
// factorisation meet at row k, where w_k = x_k), one launch per step, every
// front of the batch in the same launch.
// A workgroup computes a 16-row x 16-column tile of the block product on
// the matrix cores (four waves split the contraction and are summed in a
// fixed order) and, for the same rows, the coupling vector the next step
// needs, so each step reads one operand vector instead of two.
#include "helm_device.h"
#include "helm_launch.h"

#include <algorithm>

namespace helm {

constexpr int SW_WAVES = 4;
constexpr int SW_CTG = 1;     // 16-column tiles per workgroup (the waves split them, then K)
constexpr int SW_GDEPTH = 2;  // 16-wide K chunks of the factor block in flight per wave
constexpr int SW_YDEPTH = 2;  // and of the coupling vector
// chunks per straight-line block of the contraction: a template parameter,
// chosen per launch as the smallest even count that covers one wave's
// chunks (at most 8), so a wave does not refill chunks it never uses

int sweep_row_tiles(int np) { return np / 16; }
int sweep_col_tiles(int S) { return ((S + 15) / 16 + SW_CTG - 1) / SW_CTG; }
int sweep_grid(int groups, int cgroups) { return 8 * ((groups * cgroups + 7) / 8); }

// coupling-vector layout of the precision (b_tiled4 for complex64)
template <typename T>
__device__ __forceinline__ size_t bt(int row, int col, int np) {
    return sizeof(T) == 4 ? b_tiled4(row, col, np) : b_tiled(row, col, np);
}

template <typename C>
__device__ __forceinline__ C conj_if(C v, bool c) {
    if (c) v.y = -v.y;
    return v;
}

// y = b_{row0} into Y0 (B-operand layout; rows >= nx and columns >= S zero)
template <typename T, bool CONJB>
__global__ __launch_bounds__(256) void k_sweep_init(const SweepTab* __restrict__ tab, int n) {
    using C = typename CT<T>::c;
    const int ci = find_chain(tab->c, n, blockIdx.x, [](const SweepInfo& c) { return c.itile0; });
    const SweepInfo d = load_entry(tab->c, ci);
    const int s16 = (d.S + 15) & ~15;
    const int64_t e = (int64_t)(blockIdx.x - d.itile0) * 256 + threadIdx.x;
    if (e >= (int64_t)d.np * s16) return;
    const int s = (int)(e / d.np), k = (int)(e % d.np);
    C v = mk<C>(0.0, 0.0);
    if (k < d.nx && s < d.S)
        v = conj_if(gld((const C*)d.B + (size_t)s * d.ldb + (size_t)d.row0 * d.nx + k), CONJB);
    gst((C*)d.Y0 + bt<T>(k, s, d.np), v);
}

// One workgroup per 16-row tile of a front's block row and group of SW_CTG
// 16-column tiles of the right-hand sides: the product G_j(rows) Y(columns)
// on the matrix cores, three real products per complex one (Gauss's form:
// Gr Yr, Gi Yi and (Gr + Gi)(Yr + Yi), in separate accumulators).  The waves share out the column tiles and split the
// contraction; the parts are summed in a fixed order through LDS.  Each wave
// streams its operands with SW_DEPTH chunks of 16 in flight, and several
// workgroups per compute unit hide the rest of the latency.
template <typename T, bool FWD, bool CONJB, int SW_UNROLL>
__global__ __launch_bounds__(64 * SW_WAVES) void k_sweep(int n, int tstep, int groups, int cgroups, int uni,
                                                        const SweepTab* __restrict__ tab) {
    using C = typename CT<T>::c;
    using V = typename CT<T>::v4;
    __shared__ T red[SW_WAVES][2][4][64];
    // XCD x (workgroup b runs on XCD b % 8) takes one contiguous range of the
    // (row tile, column tile) pairs, row tile by row tile and front by front:
    // the column tiles of a row tile share its factor rows, and the row tiles
    // of a front its coupling vectors, in one or two L2s.
    const int total = groups * cgroups, per = (total + 7) >> 3;
    const int q = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
    if (q >= total) return;
    const int g = q / cgroups, cgi = q - g * cgroups;
    // uni > 0: every front of the launch has uni row tiles
    const int ci = uni > 0 ? (int)((unsigned)g / (unsigned)uni)
                           : find_chain(tab->c, n, g, [](const SweepInfo& c) { return c.tile0; });
    const SweepInfo d = load_entry(tab->c, ci);
    if (tstep >= (FWD ? d.nfwd : d.nbwd)) return;
    const int nct = (d.S + 15) >> 4, ct0 = SW_CTG * cgi;
    if (ct0 >= nct) return;
    const int nctg = min(SW_CTG, nct - ct0);
    const int P = 4 / nctg;                       // contraction parts per column tile
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int lr = l & 15, lg = l >> 4;
    const int myct = w % nctg, part = w / nctg;
    const bool active = part < P;
    const int j = FWD ? d.row0 + d.dir * tstep : d.brow0 - d.dir * tstep;
    const int i0 = 16 * (g - d.tile0);
    const int np = d.np, nx = d.nx;
    // operand streams: this row tile of G_j and this column tile of Y, each
    // 64 consecutive elements per MFMA step (the tiled layouts)
    const C* Gt = (const C*)d.G + (size_t)j * np * np + (size_t)(i0 >> 4) * (np >> 2) * 64 + l;
    const C* Gt4 = Gt - l + 4 * l;   // complex64 layout: a lane's four values of a chunk adjacent
    // steps of one front alternate the coupling buffers: forward step t is
    // step t, backward step t is step nfwd + t of the front
    const int u = FWD ? tstep : d.nfwd + tstep;
    const C* Yin = (const C*)((u & 1) ? d.Y1 : d.Y0);
    C* Yout = (C*)((u & 1) ? d.Y0 : d.Y1);
    const int s = 16 * (ct0 + myct) + lr;
    const bool scol = s < d.S;
    const C* Yt = Yin + (size_t)(ct0 + myct) * (np >> 2) * 64 + l;
    const C* Yt4 = Yt - l + 4 * l;   // complex64 layout

    // epilogue operands (next block's right-hand side, or this block's
    // forward result), fetched before the contraction.  Forward: `more` -
    // the front continues; else a bottom front hands its vector to the top
    // front (Mout), and the top front's last step is x_k.
    const C* Bv = (const C*)d.B;
    C* X = (C*)d.X;
    const bool more = FWD && tstep + 1 < d.nfwd;
    const bool merge_in = more && d.Bm && tstep + 2 == d.nfwd;
    const bool hand_over = FWD && !more && d.Mout;
    const bool lead = active && part == 0;
    // loaded unconditionally at clamped addresses (so no load waits on
    // another), then zeroed where unused
    C pre[4];
    const bool want = lead && (FWD ? (merge_in || more || hand_over) : true);
    if (lead) {
        const int sc = min(s, d.S - 1);
        const int jr = (FWD && (more || hand_over)) ? j + d.dir : j;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ic = min(i0 + acc_row<T>(lg, e), nx - 1);
            const C* src = !FWD      ? X + (size_t)sc * d.ldx + (size_t)j * nx + ic
                           : merge_in ? (const C*)d.Bm + bt<T>(ic, sc, np)
                                      : Bv + (size_t)sc * d.ldb + (size_t)jr * nx + ic;
            pre[e] = gld(src);
        }
    }
    __builtin_amdgcn_sched_barrier(0);

    V p1, p2, p3;
#pragma unroll
    for (int e = 0; e < 4; ++e) { p1[e] = 0; p2[e] = 0; p3[e] = 0; }
    // this wave's chunks of 16 in the contraction; in MFMA step q lane group
    // lg carries k = 16 ch + 4 q + lg.  Chunk indices are clamped, so every
    // load is in range.
    const int nch = np >> 4;
    const int c_beg = active ? part * nch / P : 0, c_end = active ? (part + 1) * nch / P : 0;
    C ga[SW_GDEPTH][4], ya[SW_YDEPTH][4];
    auto gload = [&](C (&gq)[4], int c) {
        const int cc = min(c, c_end - 1);
        if constexpr (sizeof(T) == 4) {
            // complex64 blocks (a_tiled4): a lane's four values of the chunk
            // are adjacent, two 16-byte loads
            typedef float gv4f __attribute__((ext_vector_type(4)));
            const HELM_GLOBAL gv4f* p = (const HELM_GLOBAL gv4f*)(Gt4 + (size_t)cc * 256);
            const gv4f a = p[0], b = p[1];
            gq[0] = mk<C>(a.x, a.y);
            gq[1] = mk<C>(a.z, a.w);
            gq[2] = mk<C>(b.x, b.y);
            gq[3] = mk<C>(b.z, b.w);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) gq[q] = gld(Gt + (size_t)(4 * cc + q) * 64);
        }
    };
    auto yload = [&](C (&yq)[4], int c) {
        const int cc = min(c, c_end - 1);
        if constexpr (sizeof(T) == 4) {
            // complex64 coupling vectors (b_tiled4): two 16-byte loads
            typedef float gv4f __attribute__((ext_vector_type(4)));
            const HELM_GLOBAL gv4f* p = (const HELM_GLOBAL gv4f*)(Yt4 + (size_t)cc * 256);
            const gv4f a = p[0], b = p[1];
            yq[0] = mk<C>(a.x, a.y);
            yq[1] = mk<C>(a.z, a.w);
            yq[2] = mk<C>(b.x, b.y);
            yq[3] = mk<C>(b.z, b.w);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) yq[q] = gld(Yt + (size_t)(4 * cc + q) * 64);
        }
    };
    // The chunks run in straight-line blocks of SW_UNROLL, each starting
    // with empty queues: the products of a chunk past the end are skipped (a
    // wave-uniform branch) while the refills stay unconditional, so the
    // outstanding loads are the same on every path and each wait covers
    // exactly the chunk about to be used.  The factor block (from HBM) is
    // fetched SW_GDEPTH chunks ahead, the coupling vector (from L2)
    // SW_YDEPTH chunks ahead.
    for (int c0 = c_beg; c0 < c_end; c0 += SW_UNROLL) {
#pragma unroll
        for (int v = 0; v < SW_GDEPTH; ++v) {
            gload(ga[v], c0 + v);
            if (v < SW_YDEPTH) yload(ya[v], c0 + v);
        }
#pragma unroll
        for (int u = 0; u < SW_UNROLL; ++u) {
            const int vg = u % SW_GDEPTH, vy = u % SW_YDEPTH;
            if (c0 + u < c_end) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T yr = ya[vy][q].x, yi = ya[vy][q].y;
                    const T gr = ga[vg][q].x, gi = ga[vg][q].y;
                    p1 = mfma16(gr, yr, p1);
                    p2 = mfma16(gi, yi, p2);
                    p3 = mfma16(gr + gi, yr + yi, p3);
                }
            }
            if (u + SW_GDEPTH < SW_UNROLL) gload(ga[vg], c0 + u + SW_GDEPTH);
            if (u + SW_YDEPTH < SW_UNROLL) yload(ya[vy], c0 + u + SW_YDEPTH);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = i0 + acc_row<T>(lg, e);
        if (!(want && scol && i < nx)) pre[e] = mk<C>(0.0, 0.0);
        else if (FWD && !merge_in) pre[e] = conj_if(pre[e], CONJB);
    }
    T sre[4], sim[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        sre[e] = p1[e] - p2[e];
        sim[e] = p3[e] - p1[e] - p2[e];
    }
    if (P > 1) {
#pragma unroll
        for (int e = 0; e < 4; ++e) { red[w][0][e][l] = sre[e]; red[w][1][e][l] = sim[e]; }
        __syncthreads();
        if (!lead) return;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            sre[e] = red[myct][0][e][l];
            sim[e] = red[myct][1][e][l];
            for (int q = 1; q < P; ++q) {
                sre[e] += red[myct + nctg * q][0][e][l];
                sim[e] += red[myct + nctg * q][1][e][l];
            }
        }
    }
    if (!lead || !scol) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = i0 + acc_row<T>(lg, e);
        const T sr = sre[e], si = sim[e];
        const T ei = (T)(i >= nx ? 0.0 : ((i == 0 || i == nx - 1) ? -0.5 * d.cz : -d.cz));
        C nxt = mk<C>(0.0, 0.0);
        if (FWD) {
            // w_j; the next step's y_{j+dir} = b_{j+dir} - E w_j; at the end
            // of a bottom front that vector goes to the top front, and at the
            // end of a top front (w_j = x_j) both backward sweeps start with E x_j
            if (i < nx) gst(X + (size_t)s * d.ldx + (size_t)j * nx + i, mk<C>(sr, si));
            if (more || hand_over) {
                if (i < nx) nxt = mk<C>(pre[e].x - ei * sr, pre[e].y - ei * si);
                if (hand_over) {
                    gst((C*)d.Mout + bt<T>(i, s, np), nxt);
                    continue;
                }
            } else {
                nxt = mk<C>(ei * sr, ei * si);
                if (d.Zp) gst((C*)d.Zp + bt<T>(i, s, np), nxt);
            }
        } else {
            // x_j = w_j - G_j z_j; the next step's z = E x_j
            if (i < nx) {
                const C xn = mk<C>(pre[e].x - sr, pre[e].y - si);
                gst(X + (size_t)s * d.ldx + (size_t)j * nx + i, xn);
                nxt = mk<C>(ei * xn.x, ei * xn.y);
            }
        }
        gst(Yout + bt<T>(i, s, np), nxt);
    }
}

void launch_sweep_init(const SweepTab* dtab, int n, int total, bool fp32, bool conj_b, hipStream_t st) {
    if (fp32) {
        if (conj_b) hipLaunchKernelGGL((k_sweep_init<float, true>), dim3(total), dim3(256), 0, st, dtab, n);
        else hipLaunchKernelGGL((k_sweep_init<float, false>), dim3(total), dim3(256), 0, st, dtab, n);
    } else {
        if (conj_b) hipLaunchKernelGGL((k_sweep_init<double, true>), dim3(total), dim3(256), 0, st, dtab, n);
        else hipLaunchKernelGGL((k_sweep_init<double, false>), dim3(total), dim3(256), 0, st, dtab, n);
    }
}

int sweep_uniform(const SweepTab& tab, int n) {
    int uni = sweep_row_tiles(tab.c[0].np);
    for (int q = 0; q < n; ++q)
        if (tab.c[q].tile0 != q * uni || sweep_row_tiles(tab.c[q].np) != uni) uni = 0;
    return uni;
}

int sweep_unroll(int np_max) {
    const int per_wave = ((np_max >> 4) + SW_WAVES - 1) / SW_WAVES;
    return std::min(8, (per_wave + 1) & ~1);
}

template <int U>
static void launch_sweep_u(const SweepTab* dtab, int n, int t, int uni, int groups, int st, bool fp32, bool forward,
                           bool conj_b, hipStream_t st_) {
    const dim3 grid(sweep_grid(groups, st)), block(64 * SW_WAVES);
    if (fp32) {
        if (forward) {
            if (conj_b) hipLaunchKernelGGL((k_sweep<float, true, true, U>), grid, block, 0, st_, n, t, groups, st, uni, dtab);
            else hipLaunchKernelGGL((k_sweep<float, true, false, U>), grid, block, 0, st_, n, t, groups, st, uni, dtab);
        } else hipLaunchKernelGGL((k_sweep<float, false, false, U>), grid, block, 0, st_, n, t, groups, st, uni, dtab);
    } else {
        if (forward) {
            if (conj_b) hipLaunchKernelGGL((k_sweep<double, true, true, U>), grid, block, 0, st_, n, t, groups, st, uni, dtab);
            else hipLaunchKernelGGL((k_sweep<double, true, false, U>), grid, block, 0, st_, n, t, groups, st, uni, dtab);
        } else hipLaunchKernelGGL((k_sweep<double, false, false, U>), grid, block, 0, st_, n, t, groups, st, uni, dtab);
    }
}

void launch_sweep(const SweepTab* dtab, int n, int t, int uni, int unroll, int groups, int st, bool fp32, bool forward,
                  bool conj_b, hipStream_t st_) {
    switch (unroll) {
        case 2: launch_sweep_u<2>(dtab, n, t, uni, groups, st, fp32, forward, conj_b, st_); break;
        case 4: launch_sweep_u<4>(dtab, n, t, uni, groups, st, fp32, forward, conj_b, st_); break;
        case 6: launch_sweep_u<6>(dtab, n, t, uni, groups, st, fp32, forward, conj_b, st_); break;
        default: launch_sweep_u<8>(dtab, n, t, uni, groups, st, fp32, forward, conj_b, st_); break;
    }
}

}  // namespace helm
