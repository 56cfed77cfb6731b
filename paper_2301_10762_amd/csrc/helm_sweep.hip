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

namespace helm {

constexpr int SW_TILE_S = 16;
constexpr int SW_WAVES = 8;

int sweep_row_tiles(int np) { return np / 16; }
int sweep_col_tiles(int S) { return (S + SW_TILE_S - 1) / SW_TILE_S; }
int sweep_grid(int groups, int st) { return 8 * ((groups + 7) / 8) * st; }

template <typename C>
__device__ __forceinline__ C conj_if(C v, bool c) {
    if (c) v.y = -v.y;
    return v;
}

// y = b_{row0} (rows >= nx zero)
template <typename T, bool CONJB>
__global__ __launch_bounds__(256) void k_sweep_init(const SweepInfo* tab, int n) {
    using C = typename CT<T>::c;
    const int ci = find_chain(tab, n, blockIdx.x, [](const SweepInfo& c) { return c.itile0; });
    const SweepInfo& d = tab[ci];
    const int64_t e = (int64_t)(blockIdx.x - d.itile0) * 256 + threadIdx.x;
    if (e >= (int64_t)d.np * d.S) return;
    const int s = (int)(e / d.np), k = (int)(e % d.np);
    C v = mk<C>(0.0, 0.0);
    if (k < d.nx) v = conj_if(((const C*)d.B)[(size_t)s * d.ldb + (size_t)d.row0 * d.nx + k], CONJB);
    ((C*)d.Y0)[e] = v;
}

// Workgroups are numbered so that the column tiles of one row tile run on
// the same XCD (consecutive workgroups go to consecutive XCDs): the rows of
// G_j they share are then read once into that XCD's L2.
template <typename T, bool FWD, bool CONJB>
__global__ __launch_bounds__(64 * SW_WAVES) void k_sweep(const SweepInfo* tab, int n, int tstep, int groups,
                                                        int st) {
    using C = typename CT<T>::c;
    using V = typename CT<T>::v4;
    __shared__ T red[SW_WAVES][2][4][64];
    const int b = blockIdx.x, xcd = b & 7, slot = b >> 3;
    const int g = (slot / st) * 8 + xcd, sidx = slot % st;
    if (g >= groups) return;
    const int ci = find_chain(tab, n, g, [](const SweepInfo& c) { return c.tile0; });
    const SweepInfo& d = tab[ci];
    if (sidx >= d.tiles_s) return;
    if (tstep >= (FWD ? d.nfwd : d.nbwd)) return;
    const int j = FWD ? d.row0 + d.dir * tstep : d.brow0 - d.dir * tstep;
    const int i0 = 16 * (g - d.tile0), s0 = SW_TILE_S * sidx;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int lr = l & 15, lg = l >> 4;
    const int np = d.np, nx = d.nx;
    const C* G = (const C*)d.G + (size_t)j * np * np + (size_t)(i0 + lr) * np;
    // steps of one front alternate the coupling buffers: forward step t is
    // step t, backward step t is step nfwd + t of the front
    const int u = FWD ? tstep : d.nfwd + tstep;
    const C* Yin = (const C*)((u & 1) ? d.Y1 : d.Y0);
    C* Yout = (C*)((u & 1) ? d.Y0 : d.Y1);
    const int s = s0 + lr;
    const bool scol = s < d.S;
    const C* y = Yin + (size_t)(scol ? s : 0) * np;

    // epilogue operands of wave 0 (next block's right-hand side, or this
    // block's forward result), fetched before the contraction.  Forward:
    // `more` - the front continues; else a bottom front hands its vector to
    // the top front (Mout), and the top front's last step is x_k.
    const C* Bv = (const C*)d.B;
    C* X = (C*)d.X;
    const bool more = FWD && tstep + 1 < d.nfwd;
    const bool merge_in = more && d.Bm && tstep + 2 == d.nfwd;
    const bool hand_over = FWD && !more && d.Mout;
    C pre[4];
    if (w == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = i0 + acc_row<T>(lg, e);
            pre[e] = mk<C>(0.0, 0.0);
            if (scol && i < nx) {
                if (FWD) {
                    if (merge_in) pre[e] = ((const C*)d.Bm)[(size_t)s * np + i];
                    else if (more || hand_over)
                        pre[e] = conj_if(Bv[(size_t)s * d.ldb + (size_t)(j + d.dir) * nx + i], CONJB);
                } else {
                    pre[e] = X[(size_t)s * d.ldx + (size_t)j * nx + i];
                }
            }
        }
    }

    V cr, cim;
#pragma unroll
    for (int e = 0; e < 4; ++e) { cr[e] = 0; cim[e] = 0; }
    // this wave's 16-column chunks of the contraction: w, w + W, w + 2W, ...;
    // two chunks' operands are loaded before they are multiplied.  In MFMA
    // step q, lane group g carries k = 16 ch + 4 q + g, so each load
    // instruction reads 64 contiguous bytes per four lanes.
    const int nch = np / 16;
    for (int base = w; base < nch; base += 2 * SW_WAVES) {
        C ga[2][4], ya[2][4];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int ch = base + c * SW_WAVES;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 16 * ch + 4 * q + lg;
                ga[c][q] = ch < nch ? G[k] : mk<C>(0.0, 0.0);
                ya[c][q] = (ch < nch && scol) ? y[k] : mk<C>(0.0, 0.0);
            }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (base + c * SW_WAVES < nch) {
#pragma unroll
                for (int q = 0; q < 4; ++q) cmfma<T, V>(cr, cim, ga[c][q].x, ga[c][q].y, ya[c][q].x, ya[c][q].y);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) { red[w][0][e][l] = cr[e]; red[w][1][e][l] = cim[e]; }
    __syncthreads();
    if (w != 0 || !scol) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = i0 + acc_row<T>(lg, e);
        T sr = red[0][0][e][l], si = red[0][1][e][l];
#pragma unroll
        for (int q = 1; q < SW_WAVES; ++q) { sr += red[q][0][e][l]; si += red[q][1][e][l]; }
        const T ei = (T)(i >= nx ? 0.0 : ((i == 0 || i == nx - 1) ? -0.5 * d.cz : -d.cz));
        C nxt = mk<C>(0.0, 0.0);
        if (FWD) {
            // w_j; the next step's y_{j+dir} = b_{j+dir} - E w_j; at the end
            // of a bottom front that vector goes to the top front, and at the
            // end of a top front (w_j = x_j) both backward sweeps start with E x_j
            if (i < nx) X[(size_t)s * d.ldx + (size_t)j * nx + i] = mk<C>(sr, si);
            if (more || hand_over) {
                if (i < nx) nxt = mk<C>(pre[e].x - ei * sr, pre[e].y - ei * si);
                if (hand_over) {
                    ((C*)d.Mout)[(size_t)s * np + i] = nxt;
                    continue;
                }
            } else {
                nxt = mk<C>(ei * sr, ei * si);
                if (d.Zp) ((C*)d.Zp)[(size_t)s * np + i] = nxt;
            }
        } else {
            // x_j = w_j - G_j z_j; the next step's z = E x_j
            if (i < nx) {
                const C xn = mk<C>(pre[e].x - sr, pre[e].y - si);
                X[(size_t)s * d.ldx + (size_t)j * nx + i] = xn;
                nxt = mk<C>(ei * xn.x, ei * xn.y);
            }
        }
        Yout[(size_t)s * np + i] = nxt;
    }
}

void launch_sweep_init(const SweepInfo* tab, int n, int total, bool fp32, bool conj_b, hipStream_t st) {
    if (fp32) {
        if (conj_b) hipLaunchKernelGGL((k_sweep_init<float, true>), dim3(total), dim3(256), 0, st, tab, n);
        else hipLaunchKernelGGL((k_sweep_init<float, false>), dim3(total), dim3(256), 0, st, tab, n);
    } else {
        if (conj_b) hipLaunchKernelGGL((k_sweep_init<double, true>), dim3(total), dim3(256), 0, st, tab, n);
        else hipLaunchKernelGGL((k_sweep_init<double, false>), dim3(total), dim3(256), 0, st, tab, n);
    }
}

void launch_sweep(const SweepInfo* tab, int n, int t, int groups, int st, bool fp32, bool forward, bool conj_b,
                  hipStream_t st_) {
    const dim3 grid(sweep_grid(groups, st)), block(64 * SW_WAVES);
    if (fp32) {
        if (forward) {
            if (conj_b) hipLaunchKernelGGL((k_sweep<float, true, true>), grid, block, 0, st_, tab, n, t, groups, st);
            else hipLaunchKernelGGL((k_sweep<float, true, false>), grid, block, 0, st_, tab, n, t, groups, st);
        } else hipLaunchKernelGGL((k_sweep<float, false, false>), grid, block, 0, st_, tab, n, t, groups, st);
    } else {
        if (forward) {
            if (conj_b) hipLaunchKernelGGL((k_sweep<double, true, true>), grid, block, 0, st_, tab, n, t, groups, st);
            else hipLaunchKernelGGL((k_sweep<double, true, false>), grid, block, 0, st_, tab, n, t, groups, st);
        } else hipLaunchKernelGGL((k_sweep<double, false, false>), grid, block, 0, st_, tab, n, t, groups, st);
    }
}

}  // namespace helm
