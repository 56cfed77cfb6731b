// Host side of libhelm: factor handles, batched block-chain drivers, solves
// with FP64 iterative refinement, and the misfit / gradient / Gauss-Newton
// drivers.  Every arithmetic step runs in the kernels of helm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cmath>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "helm.h"
#include "helm_launch.h"

using namespace helm;

struct helm_factor_s {
    helm_grid g;
    int np;
    int prec;
    double omega;
    void* G;       // nz * np * np complex (16 B for FP64, 8 B for FP32)
    double* m;     // device copy of the model
    size_t bytes;
    size_t gbytes;    // size of G
    hipStream_t st;   // the stream it was made on (its memory is released there)
    // last use on every other stream a solve ran it on (an event each); at
    // release the factor's own stream waits for them, so the memory is not
    // handed out again before those solves end, and no host wait is needed
    std::mutex mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
};

// Record that the factors of a solve were used on stream st.
void note_use(helm_factor_s* f, hipStream_t st) {
    if (!f || st == f->st) return;
    std::lock_guard<std::mutex> lk(f->mu);
    for (auto& u : f->uses)
        if (u.first == st) {
            (void)hipEventRecord(u.second, st);
            return;
        }
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(st);   // no event: wait for the use here instead
        return;
    }
    (void)hipEventRecord(ev, st);
    f->uses.push_back({st, ev});
}

// Lower-level state at one model for Hessian products (the appendix on
// products with the Hessian): the factors of A(m, w) for every frequency,
// the wavefields u and, when data are given, the adjoint fields lambda.
struct helm_hess_s {
    helm_grid g;
    int n_omega = 0, S = 0, Nr = 0, prec = 0;
    double tol = 0.0, alpha = 0.0, mu = 0.0;
    int full = 0;                        // 1: H1 + H2 + Gamma (data given); 0: H1 + Gamma
    std::vector<helm_factor_s*> F;       // one factorisation per frequency
    std::vector<double*> U, L;           // complex128 [S][N] per frequency (L only when full)
    // restriction R(P), device: RTAP taps per sensor (ntap used), value
    // weights and, for sensors at points, those of d/dx and d/dz; and its
    // transpose gathered per distinct node (nt nodes)
    int ntap = 1, nt = 0;
    bool at_points = false;
    int* rnode = nullptr;
    double* rw = nullptr;                // 3 planes of Nr * RTAP
    int *tnode = nullptr, *tptr = nullptr, *tq = nullptr;
    double* tw = nullptr;
    double* eps = nullptr;               // R(u' - u) = d - R u, complex128 [n_omega][S][Nr] (with data)
    double* m = nullptr;                 // device copy of the model
    hipStream_t st = nullptr;            // stream of creation (memory is released there)
    std::vector<std::pair<void*, size_t>> owned;
    // P2 = Gamma(p_alpha, p_mu) tables of the last PCG call
    double p_alpha = -1.0, p_mu = -1.0;
    double *Cx = nullptr, *Cz = nullptr, *eig = nullptr;
};

namespace {

thread_local std::string g_err;
std::atomic<int64_t> g_launches{0}, g_solves{0};

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHECK(x)                                                                      \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) return fail(HELM_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline hipStream_t S_(void* s) { return (hipStream_t)s; }
inline int pad16(int n) { return (n + 15) / 16 * 16; }
inline int64_t N_of(const helm_grid& g) { return (int64_t)g.nx * g.nz; }
inline size_t elem_bytes(int prec) { return prec == HELM_FP32_IR ? 8 : 16; }

size_t factor_bytes_of(const helm_grid& g, int prec) {
    size_t np = (size_t)pad16(g.nx);
    return np * np * (size_t)g.nz * elem_bytes(prec) + (size_t)N_of(g) * sizeof(double);
}

int check_grid(const helm_grid* g) {
    if (!g) return fail(HELM_EINVAL, "grid is NULL");
    if (g->nx < 2 || g->nz < 2) return fail(HELM_EINVAL, "grid needs nx >= 2 and nz >= 2");
    if (g->nx > 8192 || (int64_t)g->nx * g->nz > (int64_t)1 << 30)
        return fail(HELM_EINVAL, "grid too large");
    if (!(g->hx > 0.0) || !(g->hz > 0.0) || !std::isfinite(g->hx) || !std::isfinite(g->hz))
        return fail(HELM_EINVAL, "grid spacings must be positive and finite");
    return HELM_OK;
}

// The device's stream-ordered pool, from which the block cache below
// allocates, keeps memory released to it for reuse.
void keep_pool_memory() {
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        hipMemPool_t pool;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
    });
}

// Device memory of factors and scratch goes through a small cache of freed
// blocks.  A released block keeps an event recorded on the stream that last
// used it; a later request of about the same size on the same device takes
// it when that use is in its own stream's order or already finished, so a
// factorisation or a refinement step does not pay for a fresh allocation or
// a release (each a driver call of tens to hundreds of microseconds for
// large blocks).
// Blocks beyond the cache limit are released to the device's stream-ordered
// pool, oldest first, once their last use has finished.
struct DevCache {
    struct Blk {
        void* p;
        size_t bytes;
        int dev;
        hipEvent_t ready;
        hipStream_t st;   // the stream of the block's last use
    };
    std::mutex mu;
    std::vector<Blk> free;   // oldest first
    size_t held = 0;
    size_t limit = (size_t)32 << 30;

    static size_t rounded(size_t bytes) {
        if (bytes == 0) bytes = 16;
        const size_t q = bytes <= ((size_t)1 << 20) ? 256 : ((size_t)2 << 20);
        return (bytes + q - 1) / q * q;
    }
    void evict_locked(size_t keep) {
        while (held > keep && !free.empty()) {
            Blk b = free.front();
            free.erase(free.begin());
            held -= b.bytes;
            (void)hipEventSynchronize(b.ready);
            (void)hipEventDestroy(b.ready);
            (void)hipFreeAsync(b.p, nullptr);
        }
    }
    hipError_t get(void** out, size_t bytes, hipStream_t st) {
        const size_t rb = rounded(bytes);
        int dev = 0;
        (void)hipGetDevice(&dev);
        {
            // Candidates, best first: last used on this stream (already in
            // order), then last used elsewhere but finished (no wait); a block
            // whose last use on another stream is still queued is not taken
            // (the wait would chain this stream behind that work, e.g. one
            // serving lane behind another), a fresh block is allocated.
            std::lock_guard<std::mutex> lk(mu);
            int best = -1, best_rank = 3;
            for (int i = 0; i < (int)free.size(); ++i) {
                const Blk& b = free[i];
                if (b.dev != dev || b.bytes < rb || b.bytes > rb + rb / 4) continue;
                const int rank = b.st == st ? 0 : (hipEventQuery(b.ready) == hipSuccess ? 1 : 2);
                if (rank == 2) continue;
                if (rank < best_rank || (rank == best_rank && b.bytes < free[best].bytes)) {
                    best = i;
                    best_rank = rank;
                }
            }
            if (best >= 0) {
                Blk b = free[best];
                free.erase(free.begin() + best);
                held -= b.bytes;
                (void)hipEventDestroy(b.ready);
                *out = b.p;
                return hipSuccess;
            }
        }
        hipError_t e = hipMallocAsync(out, rb, st);
        if (e != hipSuccess) {
            // give the cached blocks back to the pool and try once more
            (void)hipGetLastError();
            {
                std::lock_guard<std::mutex> lk(mu);
                evict_locked(0);
            }
            e = hipMallocAsync(out, rb, st);
        }
        return e;
    }
    void put(void* p, size_t bytes, hipStream_t st) {
        if (!p) return;
        Blk b{p, rounded(bytes), 0, nullptr, st};
        (void)hipGetDevice(&b.dev);
        if (hipEventCreateWithFlags(&b.ready, hipEventDisableTiming) != hipSuccess) {
            (void)hipFreeAsync(p, st);
            return;
        }
        (void)hipEventRecord(b.ready, st);
        std::lock_guard<std::mutex> lk(mu);
        free.push_back(b);
        held += b.bytes;
        evict_locked(limit);
    }
    size_t set_limit(size_t bytes) {
        std::lock_guard<std::mutex> lk(mu);
        const size_t old = limit;
        limit = bytes;
        evict_locked(limit);
        return old;
    }
    size_t cached() {
        std::lock_guard<std::mutex> lk(mu);
        return held;
    }
};
DevCache g_cache;

// scratch memory, returned to the cache on scope exit (after the work that
// uses it, in stream order)
inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// A fixed device region lent to the Scratch objects of one call: bump
// allocation in 256-byte steps, given back in LIFO order as the Scratch
// scopes end.  While an Arena is installed on a thread (ArenaScope), every
// Scratch of that thread takes its memory from it and none from the cache.
struct Arena {
    char* base;
    size_t cap, used;
};
thread_local Arena* g_arena = nullptr;
struct ArenaScope {
    Arena* prev;
    explicit ArenaScope(Arena* a) : prev(g_arena) { g_arena = a; }
    ~ArenaScope() { g_arena = prev; }
};

struct Scratch {
    hipStream_t st;
    std::vector<std::pair<void*, size_t>> ptrs;
    Arena* arena;
    size_t mark;
    explicit Scratch(hipStream_t s) : st(s), arena(g_arena), mark(g_arena ? g_arena->used : 0) {}
    ~Scratch() {
        if (arena) {
            arena->used = mark;
            return;
        }
        for (auto& pb : ptrs) g_cache.put(pb.first, pb.second, st);
    }
    template <typename T>
    int get(T** out, size_t bytes) {
        if (arena) {
            const size_t off = al256(arena->used);
            if (off + bytes > arena->cap) return fail(HELM_ENOMEM, "scratch beyond the fixed region");
            arena->used = off + bytes;
            *out = (T*)(arena->base + off);
            return HELM_OK;
        }
        void* p = nullptr;
        hipError_t e = g_cache.get(&p, bytes, st);
        if (e != hipSuccess) return fail(HELM_ENOMEM, std::string("scratch allocation failed: ") + hipGetErrorString(e));
        ptrs.emplace_back(p, bytes);
        *out = (T*)p;
        return HELM_OK;
    }
};

// Optional live timing of the dominant kernels with HIP events: each run of
// back-to-back launches of one kind on a stream (the panel steps of a
// factorisation group, the steps of one forward or one backward sweep) is
// bracketed by two events on that stream; the elapsed time is booked with
// the number of launches in the run.
struct KernelTimer {
    std::mutex mu;
    int enabled = 0;
    struct Pair {
        int kind;
        int64_t launches;
        hipEvent_t a, b;
    };
    std::vector<Pair> pending;
    double total_ms[3] = {0, 0, 0};
    int64_t count[3] = {0, 0, 0};
    bool begin(int kind, hipStream_t st, Pair* p) {
        if (!enabled) return false;
        p->kind = kind;
        if (hipEventCreate(&p->a) != hipSuccess) return false;
        if (hipEventCreate(&p->b) != hipSuccess) {
            (void)hipEventDestroy(p->a);
            return false;
        }
        (void)hipEventRecord(p->a, st);
        return true;
    }
    void end(Pair& p, int64_t launches, hipStream_t st) {
        (void)hipEventRecord(p.b, st);
        p.launches = launches;
        std::lock_guard<std::mutex> lk(mu);
        pending.push_back(p);
    }
    void drain() {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                total_ms[p.kind] += ms;
                count[p.kind] += p.launches;
            }
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        pending.clear();
    }
};
KernelTimer g_timer;
int g_force_pivot = 0;   // 1: always invert diagonal tiles with partial pivoting

Coef coef_of(const helm_factor_s* f) {
    Coef c;
    c.m = f->m;
    c.omega = f->omega;
    c.hx = f->g.hx;
    c.hz = f->g.hz;
    c.nx = f->g.nx;
    c.nz = f->g.nz;
    return c;
}

// m_k > 0 and finite for every node (m in R^M_+) of each of `count`
// models; one synchronisation for all
int check_models(int count, const double* const* ms, const int64_t* ns, hipStream_t st) {
    Scratch sc(st);
    int* flag;
    int rc = sc.get(&flag, sizeof(int));
    if (rc) return rc;
    launch_zero(flag, sizeof(int), st);
    for (int c = 0; c < count; ++c) launch_check_model(ms[c], ns[c], flag, st);
    g_launches += 1 + count;
    int h = 0;
    HIPCHECK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (h) return fail(HELM_EINVAL, "model must be finite and positive at every node");
    return HELM_OK;
}
int check_model(const double* m, int64_t n, hipStream_t st) { return check_models(1, &m, &n, st); }

// ------------------------------------------------------------ factorisation --
// Factor a group of at most MAXB / 2 systems of one precision in lockstep,
// each as a top and (when nz >= 4) a bottom front: one initial launch, then
// one launch per panel step.  With pivot == 0 the diagonal tiles are
// inverted with diagonal pivots; *needs_pivot reports a front that met a
// pivot below the tolerance (the caller refactors the group).
constexpr int MAXF = MAXB / 2;   // systems per factorisation or sweep group

int factor_group(helm_factor_s* const* fs, int n, int pivot, hipStream_t st, bool* needs_pivot) {
    *needs_pivot = false;
    const bool fp32 = fs[0]->prec == HELM_FP32_IR;
    const size_t es = elem_bytes(fs[0]->prec);
    Scratch sc(st);
    ChainTab ctab;
    std::memset(&ctab, 0, sizeof(ctab));
    ChainInfo* tab = ctab.c;
    for (int c = 0; c < MAXB; ++c) tab[c].itile0 = tab[c].ftile0 = INT32_MAX;
    int utot = 0, itot = 0, Tmax = 0, nf = 0;
    size_t buf = 0;
    for (int c = 0; c < n; ++c) {
        // per system: two fronts of (P0, P1, two tile slots) and the merge
        // block, each rounded up to 256 bytes
        const size_t n2 = (size_t)fs[c]->np * fs[c]->np;
        buf += 2 * (2 * n2 + 2 * (size_t)KB * KB) * es + n2 * es + 8 * 256;
    }
    char* arena;
    int rc = sc.get(&arena, buf);
    if (rc) return rc;
    int* status;
    if ((rc = sc.get(&status, sizeof(int) * 4 * 2 * n))) return rc;
    launch_zero(status, sizeof(int) * 4 * 2 * n, st);
    ChainTab* dtab;
    if ((rc = sc.get(&dtab, sizeof(ChainTab)))) return rc;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void* p = arena + off;
        off = (off + bytes + 255) / 256 * 256;
        return p;
    };
    std::vector<int> owner;
    for (int c = 0; c < n; ++c) {
        helm_factor_s* f = fs[c];
        const size_t n2 = (size_t)f->np * f->np;
        const int nz = f->g.nz, k = twist_row(nz);
        const bool bottom = k < nz - 1;
        void* merge = bottom ? take(n2 * es) : nullptr;
        for (int side = 0; side < (bottom ? 2 : 1); ++side) {
            ChainInfo& ci = tab[nf];
            ci.G = f->G;
            ci.P0 = take(n2 * es);
            ci.P1 = take(n2 * es);
            ci.Tb = take(2 * (size_t)KB * KB * es);
            ci.status = status + 4 * nf;
            ci.cf = coef_of(f);
            ci.np = f->np;
            ci.npan = (f->np + KB - 1) / KB;
            if (side == 0) {
                ci.row0 = 0;
                ci.dir = 1;
                ci.nblk = k + 1;
                ci.Ain = merge;
                ci.Aout = nullptr;
            } else {
                ci.row0 = nz - 1;
                ci.dir = -1;
                ci.nblk = nz - 1 - k;
                ci.Ain = nullptr;
                ci.Aout = merge;
            }
            ci.T = ci.npan * ci.nblk;
            ci.pivot = pivot;
            ci.ftile0 = utot - nf;   // update workgroups of the fronts before this one
            utot += factor_step_blocks(f->np);
            ci.itile0 = itot;
            itot += factor_init_blocks(f->np);
            Tmax = std::max(Tmax, ci.T);
            owner.push_back(c);
            ++nf;
        }
    }
    launch_put_chain_table(ctab, dtab, st);
    {
        KernelTimer::Pair pi;
        const bool ti = g_timer.begin(1, st, &pi);
        launch_factor_init(dtab, nf, itot, fp32, st);
        if (ti) g_timer.end(pi, 1, st);
    }
    const int uni = factor_uniform(ctab, nf);
    KernelTimer::Pair pu;
    const bool tu = g_timer.begin(0, st, &pu);
    for (int t = 0; t < Tmax; ++t) launch_factor_step(dtab, nf, t, uni, utot, fp32, st);
    if (tu) g_timer.end(pu, Tmax, st);
    g_launches += 2 + (int64_t)Tmax;
    HIPCHECK(hipGetLastError());
    std::vector<int> hs(4 * 2 * n);   // statuses (room for 2 fronts per system)
    HIPCHECK(hipMemcpyAsync(hs.data(), status, sizeof(int) * hs.size(), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    for (int c = 0; c < nf; ++c)
        if (hs[4 * c])
            return fail(HELM_ESINGULAR, "zero pivot in a diagonal tile: system " + std::to_string(owner[c]) +
                                            ", block " + std::to_string(hs[4 * c + 1]) + ", row " +
                                            std::to_string(hs[4 * c + 2]));
    for (int c = 0; c < nf; ++c)
        if (hs[4 * c + 3]) *needs_pivot = true;
    return HELM_OK;
}

void destroy(helm_factor_s* f) {
    if (!f) return;
    {
        std::lock_guard<std::mutex> lk(f->mu);
        for (auto& u : f->uses) {
            (void)hipStreamWaitEvent(f->st, u.second, 0);
            (void)hipEventDestroy(u.second);
        }
        f->uses.clear();
    }
    if (f->G) g_cache.put(f->G, f->gbytes, f->st);
    if (f->m) g_cache.put(f->m, sizeof(double) * N_of(f->g), f->st);
    delete f;
}

int factor_many(int count, const helm_grid* grids, const double* const* m_devs, const double* omegas, int prec,
                hipStream_t st, helm_factor_t* outs) {
    if (count <= 0 || !grids || !m_devs || !omegas || !outs) return fail(HELM_EINVAL, "bad batch arguments");
    if (prec != HELM_FP64 && prec != HELM_FP32_IR) return fail(HELM_EINVAL, "unknown precision");
    std::vector<int64_t> ns(count);
    for (int c = 0; c < count; ++c) {
        int rc = check_grid(&grids[c]);
        if (rc) return rc;
        if (!m_devs[c]) return fail(HELM_EINVAL, "model pointer is NULL");
        if (!std::isfinite(omegas[c]) || omegas[c] < 0.0) return fail(HELM_EINVAL, "omega must be finite and >= 0");
        ns[c] = N_of(grids[c]);
    }
    if (int rc = check_models(count, m_devs, ns.data(), st)) return rc;
    keep_pool_memory();
    std::vector<helm_factor_s*> fs(count, nullptr);
    auto cleanup = [&]() {
        for (auto* f : fs) destroy(f);
    };
    for (int c = 0; c < count; ++c) {
        helm_factor_s* f = new helm_factor_s();
        fs[c] = f;
        f->g = grids[c];
        f->np = pad16(grids[c].nx);
        f->prec = prec;
        f->omega = omegas[c];
        f->bytes = factor_bytes_of(grids[c], prec);
        f->st = st;
        size_t gb = (size_t)f->np * f->np * (size_t)grids[c].nz * elem_bytes(prec);
        f->gbytes = gb;
        if (g_cache.get(&f->G, gb, st) != hipSuccess) {
            f->G = nullptr;
            cleanup();
            return fail(HELM_ENOMEM, "factor allocation of " + std::to_string(gb) + " bytes failed");
        }
        if (g_cache.get((void**)&f->m, sizeof(double) * N_of(grids[c]), st) != hipSuccess) {
            f->m = nullptr;
            cleanup();
            return fail(HELM_ENOMEM, "model copy allocation failed");
        }
        if (hipMemcpyAsync(f->m, m_devs[c], sizeof(double) * N_of(grids[c]), hipMemcpyDeviceToDevice, st) !=
            hipSuccess) {
            cleanup();
            return fail(HELM_EDEVICE, "model copy failed");
        }
    }
    for (int c0 = 0; c0 < count; c0 += MAXF) {
        const int k = std::min(MAXF, count - c0);
        bool needs = false;
        int rc = factor_group(fs.data() + c0, k, g_force_pivot, st, &needs);
        if (rc == HELM_OK && needs) rc = factor_group(fs.data() + c0, k, 1, st, &needs);
        if (rc) {
            cleanup();
            return rc;
        }
    }
    for (int c = 0; c < count; ++c) outs[c] = fs[c];
    return HELM_OK;
}

// ----------------------------------------------------------------- sweeps --
// X = A^{-1} Y for a group of at most MAXF factors of one precision: forward
// then backward block sweeps, from both ends of each grid.  FP64: Y, X
// complex128; FP32: complex64.  With conj_b the forward sweep reads conj(Y)
// (the adjoint solve A^{-*} r = conj(A^{-1} conj r); the caller conjugates
// the result).
int sweep_group(helm_factor_s* const* fs, int n, const void* const* Ys, const int64_t* ldy, void* const* Xs,
                const int64_t* ldx, const int* Ss, bool conj_b, hipStream_t st) {
    const bool fp32 = fs[0]->prec == HELM_FP32_IR;
    const size_t es = elem_bytes(fs[0]->prec);
    Scratch sc(st);
    SweepTab stab;
    std::memset(&stab, 0, sizeof(stab));
    SweepInfo* tab = stab.c;
    for (int c = 0; c < MAXB; ++c) tab[c].tile0 = tab[c].itile0 = INT32_MAX;
    int groups = 0, st_max = 0, itot = 0, fsteps = 0, bsteps = 0, nf = 0;
    size_t buf = 0;
    auto s16 = [](int S) { return (size_t)((S + 15) & ~15); };
    for (int c = 0; c < n; ++c) buf += 5 * ((size_t)fs[c]->np * s16(Ss[c]) * es + 256);
    char* arena;
    int rc = sc.get(&arena, buf);
    if (rc) return rc;
    SweepTab* dtab;
    if ((rc = sc.get(&dtab, sizeof(SweepTab)))) return rc;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void* p = arena + off;
        off = (off + bytes + 255) / 256 * 256;
        return p;
    };
    for (int c = 0; c < n; ++c) {
        const helm_factor_s* f = fs[c];
        const size_t yb = (size_t)f->np * s16(Ss[c]) * es;
        const int nz = f->g.nz, k = twist_row(nz);
        const bool bottom = k < nz - 1;
        const int top = nf;
        for (int side = 0; side < (bottom ? 2 : 1); ++side) {
            SweepInfo& si = tab[nf++];
            si.G = f->G;
            si.B = Ys[c];
            si.X = Xs[c];
            si.Y0 = take(yb);
            si.Y1 = take(yb);
            si.ldb = ldy[c];
            si.ldx = ldx[c];
            si.S = Ss[c];
            si.nx = f->g.nx;
            si.nz = nz;
            si.np = f->np;
            si.cz = f->g.hx / f->g.hz;
            if (side == 0) {        // rows 0..k, then back from k-1 to 0
                si.row0 = 0;
                si.dir = 1;
                si.nfwd = k + 1;
                si.brow0 = k - 1;
                si.nbwd = k;
            } else {                // rows nz-1..k+1, then back from k+1 to nz-1
                si.row0 = nz - 1;
                si.dir = -1;
                si.nfwd = nz - 1 - k;
                si.brow0 = k + 1;
                si.nbwd = nz - 1 - k;
                SweepInfo& t = tab[top];
                si.Mout = take(yb);
                t.Bm = si.Mout;
                // the bottom front's first backward step reads buffer nfwd & 1
                t.Zp = (si.nfwd & 1) ? si.Y1 : si.Y0;
            }
            si.tiles_s = sweep_col_tiles(Ss[c]);
            si.tile0 = groups;
            groups += sweep_row_tiles(f->np);
            st_max = std::max(st_max, si.tiles_s);
            si.itile0 = itot;
            itot += (int)(((int64_t)f->np * (int64_t)s16(Ss[c]) + 255) / 256);
            fsteps = std::max(fsteps, si.nfwd);
            bsteps = std::max(bsteps, si.nbwd);
        }
        g_solves += Ss[c];
    }
    launch_put_sweep_table(stab, dtab, st);
    launch_sweep_init(dtab, nf, itot, fp32, conj_b, st);
    const int uni = sweep_uniform(stab, nf);
    int np_max = 16;
    for (int c = 0; c < nf; ++c) np_max = std::max(np_max, tab[c].np);
    const int unroll = sweep_unroll(np_max);
    {
        KernelTimer::Pair p;
        const bool tm = g_timer.begin(2, st, &p);
        for (int t = 0; t < fsteps; ++t) launch_sweep(dtab, nf, t, uni, unroll, groups, st_max, fp32, true, conj_b, st);
        if (tm) g_timer.end(p, fsteps, st);
    }
    if (bsteps > 0) {
        KernelTimer::Pair p;
        const bool tm = g_timer.begin(2, st, &p);
        for (int t = 0; t < bsteps; ++t) launch_sweep(dtab, nf, t, uni, unroll, groups, st_max, fp32, false, false, st);
        if (tm) g_timer.end(p, bsteps, st);
    }
    g_launches += 2 + (int64_t)fsteps + bsteps;
    HIPCHECK(hipGetLastError());
    return HELM_OK;
}

struct SolveJob {
    helm_factor_s* f;
    const double* B;   // complex128, column-major, ld
    double* X;
    int S;
    int64_t ld;
    helm_info* info;
};

// residual norms: max over columns of ||B - A X|| / ||B||; optionally writes
// r (complex128, ld N) and/or its complex64 copy (conjugated when adjoint)
int residual_norms(const helm_factor_s* f, int adjoint, const double* B, int64_t ldb, const double* X, int64_t ldx,
                   double* R, float* R32, int S, hipStream_t st, double* maxrel) {
    Scratch sc(st);
    const int64_t N = N_of(f->g);
    const int nblk = (int)((N + 255) / 256);
    double *partial, *norms;
    int rc = sc.get(&partial, sizeof(double) * 2 * (size_t)nblk * S);
    if (rc) return rc;
    if ((rc = sc.get(&norms, sizeof(double) * 2 * S))) return rc;
    launch_residual(coef_of(f), adjoint, B, ldb, X, ldx, R, N, R32, S, partial, nblk, st);
    launch_norms_finish(partial, nblk, S, norms, st);
    g_launches += 2;
    std::vector<double> h(2 * S);
    HIPCHECK(hipMemcpyAsync(h.data(), norms, sizeof(double) * 2 * S, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    double mx = 0.0;
    for (int s = 0; s < S; ++s) {
        double rr = std::sqrt(h[2 * s]), bb = std::sqrt(h[2 * s + 1]);
        double rel = bb > 0.0 ? rr / bb : (rr > 0.0 ? INFINITY : 0.0);
        if (!(rel <= mx)) mx = rel;   // NaN propagates
    }
    *maxrel = mx;
    return HELM_OK;
}

// The same for several (factor, B, X) at once: every residual is launched,
// then one synchronisation brings all norms back.  maxrel[c] per request.
struct ResidualReq {
    const helm_factor_s* f;
    const double* B;
    int64_t ldb;
    const double* X;
    int64_t ldx;
    double* R;      // r (complex128, ld N) or NULL
    float* R32;     // conjugated-if-adjoint complex64 copy of r, or NULL
    int S;
};
int residual_norms_batch(const std::vector<ResidualReq>& rq, int adjoint, hipStream_t st, double* maxrel) {
    const int n = (int)rq.size();
    if (n == 0) return HELM_OK;
    Scratch sc(st);
    std::vector<double*> norms(n);
    size_t tot = 0;
    for (auto& r : rq) tot += 2 * (size_t)r.S;
    std::vector<double> h(tot);
    size_t off = 0;
    for (int c = 0; c < n; ++c) {
        const ResidualReq& r = rq[c];
        const int64_t N = N_of(r.f->g);
        const int nblk = (int)((N + 255) / 256);
        double* partial;
        int rc = sc.get(&partial, sizeof(double) * 2 * (size_t)nblk * r.S);
        if (rc) return rc;
        if ((rc = sc.get(&norms[c], sizeof(double) * 2 * r.S))) return rc;
        launch_residual(coef_of(r.f), adjoint, r.B, r.ldb, r.X, r.ldx, r.R, N, r.R32, r.S, partial, nblk, st);
        launch_norms_finish(partial, nblk, r.S, norms[c], st);
        g_launches += 2;
        HIPCHECK(hipMemcpyAsync(h.data() + off, norms[c], sizeof(double) * 2 * r.S, hipMemcpyDeviceToHost, st));
        off += 2 * (size_t)r.S;
    }
    HIPCHECK(hipStreamSynchronize(st));
    off = 0;
    for (int c = 0; c < n; ++c) {
        double mx = 0.0;
        for (int s = 0; s < rq[c].S; ++s) {
            double rr = std::sqrt(h[off + 2 * s]), bb = std::sqrt(h[off + 2 * s + 1]);
            double rel = bb > 0.0 ? rr / bb : (rr > 0.0 ? INFINITY : 0.0);
            if (!(rel <= mx)) mx = rel;   // NaN propagates
        }
        maxrel[c] = mx;
        off += 2 * (size_t)rq[c].S;
    }
    return HELM_OK;
}

constexpr int MAX_IR = 10;

// Solve a group of jobs that share one precision.
int solve_jobs_on(std::vector<SolveJob>& jobs, bool adjoint, double tol, hipStream_t st);

int solve_jobs(std::vector<SolveJob>& jobs, bool adjoint, double tol, hipStream_t st) {
    const int rc = solve_jobs_on(jobs, adjoint, tol, st);
    for (auto& jb : jobs) note_use(jb.f, st);
    return rc;
}

int solve_jobs_on(std::vector<SolveJob>& jobs, bool adjoint, double tol, hipStream_t st) {
    const int n = (int)jobs.size();
    if (n == 0) return HELM_OK;
    const bool fp32 = jobs[0].f->prec == HELM_FP32_IR;
    for (auto& jb : jobs) {
        if (jb.info) {
            jb.info->ir_iters = 0;
            jb.info->max_relres = -1.0;
            jb.info->bad_block = -1;
            jb.info->bad_row = -1;
            jb.info->solves = 0;
        }
    }
    std::vector<helm_factor_s*> fs(n);
    for (int c = 0; c < n; ++c) fs[c] = jobs[c].f;
    if (!fp32) {
        std::vector<const void*> Ys(n);
        std::vector<void*> Xs(n);
        std::vector<int64_t> ldy(n), ldx(n);
        std::vector<int> Ss(n);
        for (int c = 0; c < n; ++c) {
            Ys[c] = jobs[c].B;
            Xs[c] = jobs[c].X;
            ldy[c] = ldx[c] = jobs[c].ld;
            Ss[c] = jobs[c].S;
        }
        for (int c0 = 0; c0 < n; c0 += MAXF) {
            int k = std::min(MAXF, n - c0);
            int rc = sweep_group(fs.data() + c0, k, Ys.data() + c0, ldy.data() + c0, Xs.data() + c0, ldx.data() + c0,
                                 Ss.data() + c0, adjoint, st);
            if (rc) return rc;
        }
        for (int c = 0; c < n; ++c) {
            if (adjoint) {
                launch_conj_inplace(jobs[c].X, jobs[c].ld, N_of(jobs[c].f->g), jobs[c].S, st);
                g_launches += 1;
            }
            if (jobs[c].info) jobs[c].info->solves = jobs[c].S;
        }
        if (tol <= 0.0) return HELM_OK;
        // measure all jobs at once; refine in FP64 those above tol
        std::vector<ResidualReq> rq;
        for (auto& jb : jobs) rq.push_back({jb.f, jb.B, jb.ld, jb.X, jb.ld, nullptr, nullptr, jb.S});
        std::vector<double> first(n);
        int rc0 = residual_norms_batch(rq, adjoint ? 1 : 0, st, first.data());
        if (rc0) return rc0;
        for (int c = 0; c < n; ++c) {
            SolveJob& jb = jobs[c];
            if (first[c] <= tol) {
                if (jb.info) {
                    jb.info->ir_iters = 0;
                    jb.info->max_relres = first[c];
                    jb.info->solves = jb.S;
                }
                continue;
            }
            const int64_t N = N_of(jb.f->g);
            Scratch sc(st);
            double *R = nullptr, *D = nullptr;
            int it = 0;
            double rel = 0.0;
            for (;;) {
                if (!R) {
                    int rc = sc.get(&R, sizeof(double) * 2 * (size_t)N * jb.S);
                    if (rc) return rc;
                }
                int rc = residual_norms(jb.f, adjoint, jb.B, jb.ld, jb.X, jb.ld, R, nullptr, jb.S, st, &rel);
                if (rc) return rc;
                if (rel <= tol || it >= MAX_IR) break;
                if (!D && (rc = sc.get(&D, sizeof(double) * 2 * (size_t)N * jb.S))) return rc;
                helm_factor_s* f1[1] = {jb.f};
                const void* y1[1] = {R};
                void* x1[1] = {D};
                int64_t l1[1] = {N};
                int s1[1] = {jb.S};
                if ((rc = sweep_group(f1, 1, y1, l1, x1, l1, s1, adjoint, st))) return rc;
                if (adjoint) launch_conj_inplace(D, N, N, jb.S, st);
                launch_axpy_c128(D, N, jb.X, jb.ld, N, jb.S, st);
                g_launches += 2;
                ++it;
            }
            if (jb.info) {
                jb.info->ir_iters = it;
                jb.info->max_relres = rel;
                jb.info->solves = (int64_t)jb.S * (1 + it);
            }
            if (!(rel <= tol))
                return fail(HELM_ENOCONV, "FP64 solve residual " + std::to_string(rel) + " above tolerance");
        }
        return HELM_OK;
    }
    // FP32 factor: solve in complex64, refine in FP64.  The FP64 residual
    // is needed only as the complex64 right-hand side of the next correction
    // (and for its norm), so it is not stored in complex128.
    if (tol <= 0.0) tol = 1e-10;
    Scratch sc(st);
    std::vector<float*> Y32(n), X32(n);
    for (int c = 0; c < n; ++c) {
        const int64_t N = N_of(jobs[c].f->g);
        size_t bytes32 = sizeof(float) * 2 * (size_t)N * jobs[c].S;
        int rc = sc.get(&Y32[c], bytes32);
        if (rc) return rc;
        if ((rc = sc.get(&X32[c], bytes32))) return rc;
        launch_c128_to_c64(jobs[c].B, jobs[c].ld, Y32[c], N, N, jobs[c].S, adjoint ? 1 : 0, st);
        g_launches += 1;
    }
    std::vector<int> active(n, 1), iters(n, 0);
    std::vector<double> rels(n, 0.0);
    bool first = true;
    for (int round = 0;; ++round) {
        std::vector<helm_factor_s*> af;
        std::vector<const void*> ay;
        std::vector<void*> ax;
        std::vector<int64_t> al;
        std::vector<int> as, idx;
        for (int c = 0; c < n; ++c)
            if (active[c]) {
                af.push_back(fs[c]);
                ay.push_back(Y32[c]);
                ax.push_back(X32[c]);
                al.push_back(N_of(fs[c]->g));
                as.push_back(jobs[c].S);
                idx.push_back(c);
            }
        if (af.empty()) break;
        for (size_t c0 = 0; c0 < af.size(); c0 += MAXF) {
            int k = (int)std::min<size_t>(MAXF, af.size() - c0);
            int rc = sweep_group(af.data() + c0, k, ay.data() + c0, al.data() + c0, ax.data() + c0, al.data() + c0,
                                 as.data() + c0, false, st);
            if (rc) return rc;
        }
        // x (+)= conj?(y32); r = b - A x; y32 = conj?(r) for the next correction;
        // the residuals of all active jobs come back with one synchronisation
        std::vector<ResidualReq> rq;
        for (int c : idx) {
            const int64_t N = N_of(fs[c]->g);
            launch_c64_to_c128(X32[c], N, jobs[c].X, jobs[c].ld, N, jobs[c].S, adjoint ? 1 : 0, first ? 0 : 1, st);
            g_launches += 1;
            if (!first) iters[c] += 1;
            rq.push_back({fs[c], jobs[c].B, jobs[c].ld, jobs[c].X, jobs[c].ld, nullptr, Y32[c], jobs[c].S});
        }
        std::vector<double> rel(idx.size());
        int rc = residual_norms_batch(rq, adjoint ? 1 : 0, st, rel.data());
        if (rc) return rc;
        for (size_t q = 0; q < idx.size(); ++q) {
            const int c = idx[q];
            rels[c] = rel[q];
            if (rel[q] <= tol) active[c] = 0;
            else if (iters[c] >= MAX_IR) active[c] = 0;
        }
        first = false;
    }
    int worst = HELM_OK;
    for (int c = 0; c < n; ++c) {
        if (jobs[c].info) {
            jobs[c].info->ir_iters = iters[c];
            jobs[c].info->max_relres = rels[c];
            jobs[c].info->solves = (int64_t)jobs[c].S * (1 + iters[c]);
        }
        if (!(rels[c] <= tol)) worst = fail(HELM_ENOCONV, "refinement stopped at relative residual " +
                                                              std::to_string(rels[c]) + " > " + std::to_string(tol));
    }
    return worst;
}

// host -> device copy of caller-owned host data, complete on return
int upload_sync(void* dev, const void* src, size_t bytes, hipStream_t st) {
    HIPCHECK(hipMemcpyAsync(dev, src, bytes, hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    return HELM_OK;
}

int check_solve_args(const helm_factor_s* f, const double* B, double* X, int S, int64_t ld) {
    if (!f) return fail(HELM_EINVAL, "factor is NULL");
    if (!B || !X) return fail(HELM_EINVAL, "NULL right-hand side or solution pointer");
    if (S <= 0) return fail(HELM_EINVAL, "S must be positive");
    const int64_t N = N_of(f->g);
    if (ld < N) return fail(HELM_EINVAL, "ld must be >= nx*nz");
    const char* b0 = (const char*)B;
    const char* b1 = b0 + 16 * ((size_t)(S - 1) * ld + N);
    const char* x0 = (const char*)X;
    const char* x1 = x0 + 16 * ((size_t)(S - 1) * ld + N);
    if (x0 < b1 && b0 < x1) return fail(HELM_EINVAL, "X must not overlap B");
    return HELM_OK;
}

int check_nodes(const int32_t* nodes, int count, int64_t N, const char* what) {
    if (count > 0 && !nodes) return fail(HELM_EINVAL, std::string(what) + " list is NULL");
    for (int q = 0; q < count; ++q)
        if (nodes[q] < 0 || nodes[q] >= N)
            return fail(HELM_EINVAL, std::string(what) + " node index out of range");
    return HELM_OK;
}

// ------------------------------------------------------- Hessian products --

template <typename T>
int hess_own(helm_hess_s* h, T** out, size_t bytes) {
    void* p = nullptr;
    hipError_t e = g_cache.get(&p, bytes, h->st);
    if (e != hipSuccess) return fail(HELM_ENOMEM, std::string("allocation failed: ") + hipGetErrorString(e));
    h->owned.emplace_back(p, bytes);
    *out = (T*)p;
    return HELM_OK;
}

void hess_free(helm_hess_s* h) {
    if (!h) return;
    for (auto f : h->F) destroy(f);
    for (auto& pb : h->owned) g_cache.put(pb.first, pb.second, h->st);
    delete h;
}

// Orthonormal DCT-II matrices of sizes nx and nz and the eigenvalues of
// Gamma(alpha, mu) on that basis, uploaded (complete on return).  Angles are
// reduced exactly in integers before the cosine is taken.
int gamma_tables(int nx, int nz, double alpha, double mu, double* Cx, double* Cz, double* eig, hipStream_t st) {
    const double pi = 3.14159265358979323846;
    auto dct = [&](int n, std::vector<double>& c) {
        c.assign((size_t)n * n, 0.0);
        for (int p = 0; p < n; ++p) {
            const double sc = std::sqrt((p == 0 ? 1.0 : 2.0) / n);
            for (int i = 0; i < n; ++i) {
                const int64_t a = ((int64_t)p * (2 * i + 1)) % (4 * (int64_t)n);   // angle pi a / (2 n)
                c[(size_t)p * n + i] = sc * std::cos(pi * (double)a / (2.0 * n));
            }
        }
    };
    auto lap = [&](int n, int p) {   // (n-1)^2 * 4 sin^2(pi p / (2 n))
        const double sn = std::sin(pi * p / (2.0 * n));
        return (double)(n - 1) * (n - 1) * 4.0 * sn * sn;
    };
    std::vector<double> cx, cz, ev((size_t)nx * nz);
    dct(nx, cx);
    dct(nz, cz);
    for (int q = 0; q < nz; ++q)
        for (int p = 0; p < nx; ++p) ev[(size_t)q * nx + p] = alpha * (lap(nx, p) + lap(nz, q)) + mu;
    HIPCHECK(hipMemcpyAsync(Cx, cx.data(), sizeof(double) * cx.size(), hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(Cz, cz.data(), sizeof(double) * cz.size(), hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(eig, ev.data(), sizeof(double) * ev.size(), hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    return HELM_OK;
}

void merge_info(helm_info* into, const helm_info& a) {
    into->ir_iters = std::max(into->ir_iters, a.ir_iters);
    into->max_relres = std::max(into->max_relres, a.max_relres);
    into->solves += a.solves;
}

// A restriction R(P) on the host: RTAP taps per sensor (only the first ntap
// used), weights for the value and for d/dx, d/dz of the sensor position,
// and the transpose of the value weights gathered per distinct node.
struct HostRTab {
    int Nr = 0, ntap = 1;
    bool points = false;
    std::vector<int> node;                    // Nr * RTAP
    std::vector<double> w;                    // 3 planes of Nr * RTAP
    std::vector<int> tnode, tptr, tq;
    std::vector<double> tw;
};

// Sliding cubic along one grid line (App. "Numerical restriction operator"):
// at grid coordinate u (position / spacing) on n >= 4 nodes, the Lagrange
// cubic through the four nodes nearest to u (those of its interval and one
// on each side, moved inward at the ends).  Weights L for the value and dL
// for d/du.
void cubic_stencil(double u, int n, int* first, double L[4], double dL[4]) {
    int i = (int)std::floor(u);
    i = std::min(std::max(i, 0), n - 2);
    const int i0 = std::min(std::max(i - 1, 0), n - 4);
    const double t = u - i0, a = t, b = t - 1.0, c = t - 2.0, d = t - 3.0;
    L[0] = -(b * c * d) / 6.0;
    L[1] = (a * c * d) / 2.0;
    L[2] = -(a * b * d) / 2.0;
    L[3] = (a * b * c) / 6.0;
    dL[0] = -(c * d + b * d + b * c) / 6.0;
    dL[1] = (c * d + a * d + a * c) / 2.0;
    dL[2] = -(b * d + a * d + a * b) / 2.0;
    dL[3] = (b * c + a * c + a * b) / 6.0;
    *first = i0;
}

void rtab_transpose(HostRTab* t, int64_t N) {
    std::vector<std::vector<std::pair<int, double>>> by;   // per touched node: (sensor, weight)
    std::vector<int> slot(N, -1);
    for (int q = 0; q < t->Nr; ++q)
        for (int a = 0; a < t->ntap; ++a) {
            const double wv = t->w[(size_t)q * RTAP + a];
            if (wv == 0.0) continue;
            const int k = t->node[(size_t)q * RTAP + a];
            if (slot[k] < 0) {
                slot[k] = (int)by.size();
                t->tnode.push_back(k);
                by.emplace_back();
            }
            by[slot[k]].emplace_back(q, wv);
        }
    t->tptr.assign(1, 0);
    for (auto& lst : by) {
        for (auto& e : lst) {
            t->tq.push_back(e.first);
            t->tw.push_back(e.second);
        }
        t->tptr.push_back((int)t->tq.size());
    }
}

// sensors on nodes: one tap of weight 1 (plain sampling)
int rtab_nodes(const helm_grid& g, int Nr, const int32_t* nodes, HostRTab* t) {
    int rc = check_nodes(nodes, Nr, N_of(g), "receiver");
    if (rc) return rc;
    t->Nr = Nr;
    t->ntap = 1;
    t->node.assign((size_t)Nr * RTAP, 0);
    t->w.assign((size_t)3 * Nr * RTAP, 0.0);
    for (int q = 0; q < Nr; ++q) {
        for (int a = 0; a < RTAP; ++a) t->node[(size_t)q * RTAP + a] = nodes[q];
        t->w[(size_t)q * RTAP] = 1.0;
    }
    rtab_transpose(t, N_of(g));
    return HELM_OK;
}

// sensors at points (x, z) of the domain: the sliding bicubic, 16 taps
int rtab_points(const helm_grid& g, int Nr, const double* xz, HostRTab* t) {
    if (Nr > 0 && !xz) return fail(HELM_EINVAL, "sensor position list is NULL");
    if (g.nx < 4 || g.nz < 4) return fail(HELM_EINVAL, "sensors at points need nx, nz >= 4 (bicubic stencil)");
    const double X = g.hx * (g.nx - 1), Z = g.hz * (g.nz - 1);
    t->Nr = Nr;
    t->ntap = RTAP;
    t->points = true;
    t->node.assign((size_t)Nr * RTAP, 0);
    t->w.assign((size_t)3 * Nr * RTAP, 0.0);
    const size_t plane = (size_t)Nr * RTAP;
    for (int q = 0; q < Nr; ++q) {
        const double x = xz[2 * q], z = xz[2 * q + 1];
        if (!(x >= 0.0 && x <= X && z >= 0.0 && z <= Z))
            return fail(HELM_EINVAL, "sensor " + std::to_string(q) + " lies outside the domain");
        int i0, j0;
        double Lx[4], dLx[4], Lz[4], dLz[4];
        cubic_stencil(x / g.hx, g.nx, &i0, Lx, dLx);
        cubic_stencil(z / g.hz, g.nz, &j0, Lz, dLz);
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                const size_t e = (size_t)q * RTAP + 4 * b + a;
                t->node[e] = (j0 + b) * g.nx + i0 + a;
                t->w[e] = Lx[a] * Lz[b];
                t->w[plane + e] = dLx[a] / g.hx * Lz[b];
                t->w[2 * plane + e] = Lx[a] * dLz[b] / g.hz;
            }
    }
    rtab_transpose(t, N_of(g));
    return HELM_OK;
}

int check_points(const helm_grid& g, int n, const double* xz, const char* what) {
    if (n > 0 && !xz) return fail(HELM_EINVAL, std::string(what) + " position list is NULL");
    const double X = g.hx * (g.nx - 1), Z = g.hz * (g.nz - 1);
    for (int q = 0; q < n; ++q)
        if (!(xz[2 * q] >= 0.0 && xz[2 * q] <= X && xz[2 * q + 1] >= 0.0 && xz[2 * q + 1] <= Z))
            return fail(HELM_EINVAL, std::string(what) + " " + std::to_string(q) + " lies outside the domain");
    return HELM_OK;
}

// Factor A(m, w) for every frequency and solve for u (and, with data, for
// lambda = A^{-*} R^*(d - R u), phi and grad phi when asked for).  The
// fields stay with the returned context; the stream is synchronised.
int hess_build(const helm_grid* grid, const double* m_dev, int n_omega, const double* omegas_host,
               const double* dobs_dev, int S, const int32_t* src_host, const double* src_xz, int Nr,
               const int32_t* rec_host, const double* rec_xz, double alpha, double mu, int precision, double tol,
               hipStream_t st, double* phi_host, double* grad_dev, helm_info* info, helm_hess_s** out) {
    *out = nullptr;
    int rc = check_grid(grid);
    if (rc) return rc;
    if (n_omega <= 0 || S <= 0 || Nr <= 0 || !omegas_host || !m_dev)
        return fail(HELM_EINVAL, "bad frequency, source or receiver counts, or NULL pointers");
    if (precision != HELM_FP64 && precision != HELM_FP32_IR) return fail(HELM_EINVAL, "unknown precision");
    const int64_t N = N_of(*grid);
    if ((src_host != nullptr) == (src_xz != nullptr)) return fail(HELM_EINVAL, "give either source nodes or points");
    if ((rc = src_xz ? check_points(*grid, S, src_xz, "source") : check_nodes(src_host, S, N, "source"))) return rc;
    HostRTab rt;
    if ((rc = rec_xz ? rtab_points(*grid, Nr, rec_xz, &rt) : rtab_nodes(*grid, Nr, rec_host, &rt))) return rc;
    const bool full = dobs_dev != nullptr;
    if (full)
        for (int s = 0; s < S; ++s)
            for (int p = 0; p < Nr; ++p) {
                const double sx = src_xz ? src_xz[2 * s] : (src_host[s] % grid->nx) * grid->hx;
                const double sz = src_xz ? src_xz[2 * s + 1] : (src_host[s] / grid->nx) * grid->hz;
                const double rx = rec_xz ? rec_xz[2 * p] : (rec_host[p] % grid->nx) * grid->hx;
                const double rz = rec_xz ? rec_xz[2 * p + 1] : (rec_host[p] / grid->nx) * grid->hz;
                if (std::fabs(sx - rx) <= 1e-12 * grid->hx && std::fabs(sz - rz) <= 1e-12 * grid->hz)
                    return fail(HELM_EINVAL, "a source coincides with a receiver");
            }
    helm_hess_s* h = new helm_hess_s();
    *out = h;
    h->g = *grid;
    h->n_omega = n_omega;
    h->S = S;
    h->Nr = Nr;
    h->prec = precision;
    h->tol = tol;
    h->alpha = alpha;
    h->mu = mu;
    h->full = full ? 1 : 0;
    h->st = st;
    std::vector<helm_grid> grids(n_omega, *grid);
    std::vector<const double*> ms(n_omega, m_dev);
    h->F.assign(n_omega, nullptr);
    if ((rc = factor_many(n_omega, grids.data(), ms.data(), omegas_host, precision, st, h->F.data()))) return rc;
    h->m = h->F[0]->m;
    Scratch sc(st);
    int* dsrc = nullptr;
    double* dsxz = nullptr;
    if (src_xz) {
        if ((rc = sc.get(&dsxz, sizeof(double) * 2 * S))) return rc;
        if ((rc = upload_sync(dsxz, src_xz, sizeof(double) * 2 * S, st))) return rc;
    } else {
        if ((rc = sc.get(&dsrc, sizeof(int) * S))) return rc;
        if ((rc = upload_sync(dsrc, src_host, sizeof(int) * S, st))) return rc;
    }
    h->ntap = rt.ntap;
    h->at_points = rt.points;
    h->nt = (int)rt.tnode.size();
    if ((rc = hess_own(h, &h->rnode, sizeof(int) * rt.node.size()))) return rc;
    if ((rc = hess_own(h, &h->rw, sizeof(double) * rt.w.size()))) return rc;
    if ((rc = hess_own(h, &h->tnode, sizeof(int) * std::max<size_t>(rt.tnode.size(), 1)))) return rc;
    if ((rc = hess_own(h, &h->tptr, sizeof(int) * rt.tptr.size()))) return rc;
    if ((rc = hess_own(h, &h->tq, sizeof(int) * std::max<size_t>(rt.tq.size(), 1)))) return rc;
    if ((rc = hess_own(h, &h->tw, sizeof(double) * std::max<size_t>(rt.tw.size(), 1)))) return rc;
    if ((rc = upload_sync(h->rnode, rt.node.data(), sizeof(int) * rt.node.size(), st))) return rc;
    if ((rc = upload_sync(h->rw, rt.w.data(), sizeof(double) * rt.w.size(), st))) return rc;
    if ((rc = upload_sync(h->tptr, rt.tptr.data(), sizeof(int) * rt.tptr.size(), st))) return rc;
    if (h->nt > 0) {
        if ((rc = upload_sync(h->tnode, rt.tnode.data(), sizeof(int) * rt.tnode.size(), st))) return rc;
        if ((rc = upload_sync(h->tq, rt.tq.data(), sizeof(int) * rt.tq.size(), st))) return rc;
        if ((rc = upload_sync(h->tw, rt.tw.data(), sizeof(double) * rt.tw.size(), st))) return rc;
    }
    const size_t fb = sizeof(double) * 2 * (size_t)N * S;
    double* E;
    if ((rc = sc.get(&E, fb))) return rc;
    h->U.assign(n_omega, nullptr);
    for (int w = 0; w < n_omega; ++w)
        if ((rc = hess_own(h, &h->U[w], fb))) return rc;
    if (src_xz) {
        launch_zero(E, fb, st);
        launch_point_sources(E, N, dsxz, S, grid->nx, grid->nz, grid->hx, grid->hz, st);
        g_launches += 2;
    } else {
        launch_unit_sources(E, N, N, dsrc, S, st);
        g_launches += 1;
    }
    // forward wavefields u = A^{-1} f_s, all frequencies in one batch
    std::vector<SolveJob> jobs;
    std::vector<helm_info> infos(n_omega);
    for (int w = 0; w < n_omega; ++w) jobs.push_back({h->F[w], E, h->U[w], S, N, &infos[w]});
    if ((rc = solve_jobs(jobs, false, tol, st))) return rc;
    helm_info tot{};
    tot.bad_block = tot.bad_row = -1;
    for (auto& i1 : infos) merge_info(&tot, i1);
    if (full) {
        // residuals at the receivers, phi, adjoint sources R^* eps, then lambda
        double *eps, *phip;
        std::vector<double*> Radj(n_omega);
        if ((rc = hess_own(h, &h->eps, sizeof(double) * 2 * (size_t)Nr * S * n_omega))) return rc;
        eps = h->eps;
        if ((rc = sc.get(&phip, sizeof(double) * (size_t)S * n_omega + 8))) return rc;
        h->L.assign(n_omega, nullptr);
        for (int w = 0; w < n_omega; ++w) {
            if ((rc = hess_own(h, &h->L[w], fb))) return rc;
            if ((rc = sc.get(&Radj[w], fb))) return rc;
        }
        for (int w = 0; w < n_omega; ++w) {
            launch_misfit(h->U[w], N, dobs_dev + 2 * (size_t)w * S * Nr, h->rnode, h->rw, h->ntap, Nr, S,
                          eps + 2 * (size_t)w * S * Nr, phip + (size_t)w * S, st);
            launch_zero(Radj[w], fb, st);
            if (h->nt > 0)
                launch_restrict_adj(eps + 2 * (size_t)w * S * Nr, Nr, h->tnode, h->tptr, h->tq, h->tw, h->nt, S,
                                    Radj[w], N, st);
            g_launches += 3;
        }
        std::vector<SolveJob> ajobs;
        std::vector<helm_info> ainfos(n_omega);
        for (int w = 0; w < n_omega; ++w) ajobs.push_back({h->F[w], Radj[w], h->L[w], S, N, &ainfos[w]});
        if ((rc = solve_jobs(ajobs, true, tol, st))) return rc;
        for (auto& i2 : ainfos) merge_info(&tot, i2);
        double reg = 0.0;
        if (grad_dev) {
            launch_zero(grad_dev, sizeof(double) * N, st);
            for (int w = 0; w < n_omega; ++w) launch_grad(coef_of(h->F[w]), h->U[w], N, h->L[w], N, S, grad_dev, st);
            g_launches += 1 + n_omega;
        }
        if (grad_dev && (alpha != 0.0 || mu != 0.0)) {
            const int nblk = (int)((N + 255) / 256);
            double *part, *q;
            if ((rc = sc.get(&part, sizeof(double) * nblk))) return rc;
            if ((rc = sc.get(&q, sizeof(double)))) return rc;
            launch_gamma(m_dev, grid->nx, grid->nz, alpha, mu, grad_dev, part, nblk, st);
            launch_sum_scalar(part, nblk, q, st);
            g_launches += 2;
            HIPCHECK(hipMemcpyAsync(&reg, q, sizeof(double), hipMemcpyDeviceToHost, st));
        }
        if (phi_host) {
            std::vector<double> hp((size_t)S * n_omega);
            HIPCHECK(hipMemcpyAsync(hp.data(), phip, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
            double phi = 0.0;
            for (double v : hp) phi += v;
            *phi_host = phi + 0.5 * reg;
        }
    }
    HIPCHECK(hipStreamSynchronize(st));
    HIPCHECK(hipGetLastError());
    if (info) *info = tot;
    return HELM_OK;
}

// hv_a = H mt_a for n_dir directions, for several contexts at once (one
// direction block per context): per frequency v = A^{-1}(g mt u) for
// every source and direction, then
//   z = A^{-*}(R^* R v - conj(g) mt lambda)   (full) or A^{-*}(R^* R v),
//   hv += Re g u conj(z) - Re g v conj(lambda) - Re h mt u conj(lambda)  (full)
//   or    Re g u conj(z),
// the frequencies of all contexts batched into one forward and one adjoint
// solve (the contexts must share precision and tolerance); finally
// hv += Gamma mt.  Synchronises the stream.
int hess_apply_multi(const std::vector<helm_hess_s*>& hs, int n_dir, const std::vector<const double*>& mts,
                     const std::vector<double*>& hvs, hipStream_t st, std::vector<helm_info>* infos) {
    const int K = (int)hs.size();
    for (auto h : hs)
        if (h->prec != hs[0]->prec || h->tol != hs[0]->tol)
            return fail(HELM_EINVAL, "batched Hessian products need one precision and tolerance");
    Scratch sc(st);
    struct Part {
        std::vector<double*> W, V, Z;
        double* RV;
        std::vector<helm_info> i1, i2;
    };
    std::vector<Part> P(K);
    std::vector<SolveJob> j1, j2;
    int rc;
    for (int c = 0; c < K; ++c) {
        helm_hess_s* h = hs[c];
        const int64_t N = N_of(h->g);
        const int S = h->S, nw = h->n_omega;
        if ((int64_t)n_dir * S > 65535)
            return fail(HELM_EINVAL, "n_dir * S must not exceed 65535 (split the directions)");
        const int cols = n_dir * S;
        const size_t vb = sizeof(double) * 2 * (size_t)N * cols;
        Part& q = P[c];
        q.W.resize(nw), q.V.resize(nw), q.Z.resize(nw), q.i1.resize(nw), q.i2.resize(nw);
        if ((rc = sc.get(&q.RV, sizeof(double) * 2 * (size_t)h->Nr * cols))) return rc;
        for (int w = 0; w < nw; ++w) {
            if ((rc = sc.get(&q.W[w], vb))) return rc;
            if ((rc = sc.get(&q.V[w], vb))) return rc;
            if ((rc = sc.get(&q.Z[w], vb))) return rc;
            launch_gn_rhs(coef_of(h->F[w]), h->U[w], N, S, mts[c], n_dir, q.W[w], N, st);
            j1.push_back({h->F[w], q.W[w], q.V[w], cols, N, &q.i1[w]});
        }
        g_launches += nw;
    }
    if ((rc = solve_jobs(j1, false, hs[0]->tol, st))) return rc;
    // W now holds the right-hand side of the z solve
    for (int c = 0; c < K; ++c) {
        helm_hess_s* h = hs[c];
        const int64_t N = N_of(h->g);
        const int S = h->S, nw = h->n_omega, cols = n_dir * S;
        Part& q = P[c];
        for (int w = 0; w < nw; ++w) {
            if (h->full) launch_zeta_rhs(coef_of(h->F[w]), h->L[w], N, S, mts[c], n_dir, q.W[w], N, st);
            else launch_zero(q.W[w], sizeof(double) * 2 * (size_t)N * cols, st);
            // W += R^T R v
            launch_restrict(q.V[w], N, h->rnode, h->rw, h->ntap, h->Nr, cols, q.RV, h->Nr, st);
            if (h->nt > 0)
                launch_restrict_adj(q.RV, h->Nr, h->tnode, h->tptr, h->tq, h->tw, h->nt, cols, q.W[w], N, st);
            g_launches += 3;
            j2.push_back({h->F[w], q.W[w], q.Z[w], cols, N, &q.i2[w]});
        }
    }
    if ((rc = solve_jobs(j2, true, hs[0]->tol, st))) return rc;
    for (int c = 0; c < K; ++c) {
        helm_hess_s* h = hs[c];
        const int64_t N = N_of(h->g);
        const int S = h->S, nw = h->n_omega;
        Part& q = P[c];
        launch_zero(hvs[c], sizeof(double) * N * n_dir, st);
        for (int w = 0; w < nw; ++w) {
            if (h->full)
                launch_hv_full(coef_of(h->F[w]), h->U[w], h->L[w], N, S, q.V[w], q.Z[w], N, mts[c], n_dir, hvs[c],
                               st);
            else
                launch_hv(coef_of(h->F[w]), h->U[w], N, S, q.Z[w], N, n_dir, hvs[c], N, st);
        }
        g_launches += 1 + nw;
        if (h->alpha != 0.0 || h->mu != 0.0) {
            const int nblk = (int)((N + 255) / 256);
            double* part;
            if ((rc = sc.get(&part, sizeof(double) * nblk))) return rc;
            for (int a = 0; a < n_dir; ++a)
                launch_gamma(mts[c] + (size_t)a * N, h->g.nx, h->g.nz, h->alpha, h->mu, hvs[c] + (size_t)a * N, part,
                             nblk, st);
            g_launches += n_dir;
        }
    }
    HIPCHECK(hipStreamSynchronize(st));
    HIPCHECK(hipGetLastError());
    if (infos) {
        infos->assign(K, helm_info{});
        for (int c = 0; c < K; ++c) {
            helm_info& tot = (*infos)[c];
            tot.bad_block = tot.bad_row = -1;
            for (size_t w = 0; w < P[c].i1.size(); ++w) {
                merge_info(&tot, P[c].i1[w]);
                merge_info(&tot, P[c].i2[w]);
            }
        }
    }
    return HELM_OK;
}

int hess_apply(helm_hess_s* h, int n_dir, const double* mt, double* hv, hipStream_t st, helm_info* info) {
    std::vector<helm_info> infos;
    int rc = hess_apply_multi({h}, n_dir, {mt}, {hv}, st, &infos);
    if (rc == HELM_OK && info) *info = infos[0];
    return rc;
}

// the P2 = Gamma(p_alpha, p_mu) tables of a context, made on first use
int hess_p2_tables(helm_hess_s* h, double p_alpha, double p_mu, hipStream_t st) {
    if (h->Cx && h->p_alpha == p_alpha && h->p_mu == p_mu) return HELM_OK;
    const int nx = h->g.nx, nz = h->g.nz;
    int rc;
    if (!h->Cx) {
        if ((rc = hess_own(h, &h->Cx, sizeof(double) * nx * nx))) return rc;
        if ((rc = hess_own(h, &h->Cz, sizeof(double) * nz * nz))) return rc;
        if ((rc = hess_own(h, &h->eig, sizeof(double) * N_of(h->g)))) return rc;
    }
    // the tables were allocated on the creation stream
    HIPCHECK(hipStreamSynchronize(h->st));
    if ((rc = gamma_tables(nx, nz, p_alpha, p_mu, h->Cx, h->Cz, h->eig, st))) return rc;
    h->p_alpha = p_alpha;
    h->p_mu = p_mu;
    return HELM_OK;
}

// Preconditioned conjugate gradients for H_c x_c = b_c (eq (rho)), one
// system per context, run in lockstep so that the products with all the
// H_c share their sweep launches; P2 = Gamma(p_alpha, p_mu) (eq (P2); none
// when p_mu <= 0); each system stops once ||r_n|| <= rtol ||r_0|| (or on
// p.Hp <= 0, status 2) and leaves the lockstep.  x_c holds the start
// vector on entry.  The scalars of a step come back to the host together.
// status[c]: 0 converged, 1 iteration limit, 2 not positive definite.
int hess_pcg_multi(const std::vector<helm_hess_s*>& hs, const std::vector<const double*>& b,
                   const std::vector<double*>& x, double p_alpha, double p_mu, double rtol, int maxit,
                   hipStream_t st, int32_t* iters, double* relres, int32_t* status, std::vector<helm_info>* infos) {
    const int K = (int)hs.size();
    for (int c = 0; c < K; ++c)
        if (!b[c] || !x[c]) return fail(HELM_EINVAL, "bad pcg arguments");
    if (maxit < 0 || !(rtol >= 0.0)) return fail(HELM_EINVAL, "bad pcg arguments");
    const bool prec = p_mu > 0.0;
    if (!prec && p_alpha != 0.0) return fail(HELM_EINVAL, "P2 = Gamma(alpha, mu) needs mu > 0");
    if (prec && !(p_alpha >= 0.0)) return fail(HELM_EINVAL, "P2 = Gamma(alpha, mu) needs alpha >= 0");
    Scratch sc(st);
    std::vector<double*> r(K), z(K), p(K), q(K), T1(K), T2(K);
    double *part, *scal;
    int rc;
    int64_t Nmax = 0;
    for (auto h : hs) Nmax = std::max(Nmax, N_of(h->g));
    if ((rc = sc.get(&part, sizeof(double) * dot_blocks(Nmax)))) return rc;
    if ((rc = sc.get(&scal, sizeof(double) * K))) return rc;
    for (int c = 0; c < K; ++c) {
        const size_t vb = sizeof(double) * N_of(hs[c]->g);
        if ((rc = sc.get(&r[c], vb))) return rc;
        if ((rc = sc.get(&p[c], vb))) return rc;
        if ((rc = sc.get(&q[c], vb))) return rc;
        z[c] = r[c];
        if (prec) {
            if ((rc = sc.get(&z[c], vb))) return rc;
            if ((rc = sc.get(&T1[c], vb))) return rc;
            if ((rc = sc.get(&T2[c], vb))) return rc;
            if ((rc = hess_p2_tables(hs[c], p_alpha, p_mu, st))) return rc;
        }
    }
    // u.v for the listed systems, one synchronisation
    auto dots = [&](const std::vector<int>& cs, const std::vector<double*>& u, const std::vector<double*>& v,
                    std::vector<double>& out) -> int {
        for (size_t k = 0; k < cs.size(); ++k) {
            const int c = cs[k];
            launch_dot(u[c], v[c], N_of(hs[c]->g), part, scal + k, st);
            g_launches += 2;
        }
        std::vector<double> h(cs.size());
        HIPCHECK(hipMemcpyAsync(h.data(), scal, sizeof(double) * cs.size(), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        for (size_t k = 0; k < cs.size(); ++k) out[cs[k]] = h[k];
        return HELM_OK;
    };
    auto apply = [&](const std::vector<int>& cs, const std::vector<double*>& in) -> int {
        std::vector<helm_hess_s*> hh;
        std::vector<const double*> mm;
        std::vector<double*> oo;
        for (int c : cs) {
            hh.push_back(hs[c]);
            mm.push_back(in[c]);
            oo.push_back(q[c]);
        }
        std::vector<helm_info> ii;
        int r2 = hess_apply_multi(hh, 1, mm, oo, st, &ii);
        if (r2) return r2;
        for (size_t k = 0; k < cs.size(); ++k) merge_info(&(*infos)[cs[k]], ii[k]);
        return HELM_OK;
    };
    auto precondition = [&](const std::vector<int>& cs) {
        if (!prec) return;
        for (int c : cs) {
            launch_gamma_solve(hs[c]->Cx, hs[c]->Cz, hs[c]->eig, hs[c]->g.nx, hs[c]->g.nz, 1, r[c], z[c], T1[c],
                               T2[c], st);
            g_launches += 4;
        }
    };
    infos->assign(K, helm_info{});
    for (auto& i0 : *infos) i0.bad_block = i0.bad_row = -1;
    std::vector<double> rr0(K), rr(K), rz(K), pq(K), rz1(K), rel(K, 0.0);
    std::vector<int> all(K), it(K, 0), st_(K, 1);
    for (int c = 0; c < K; ++c) all[c] = c;
    // r = b - H x
    if ((rc = apply(all, x))) return rc;
    for (int c = 0; c < K; ++c) launch_lincomb(r[c], 1.0, b[c], -1.0, q[c], N_of(hs[c]->g), st);
    g_launches += K;
    if ((rc = dots(all, r, r, rr0))) return rc;
    std::vector<int> act;
    for (int c = 0; c < K; ++c) {
        if (rr0[c] > 0.0) {
            rel[c] = 1.0;
            act.push_back(c);
        } else {
            st_[c] = 0;
        }
    }
    precondition(act);
    for (int c : act) launch_lincomb(p[c], 1.0, z[c], 0.0, z[c], N_of(hs[c]->g), st);
    g_launches += (int)act.size();
    if ((rc = dots(act, r, z, rz))) return rc;
    for (int step = 0; step < maxit && !act.empty(); ++step) {
        if ((rc = apply(act, p))) return rc;
        if ((rc = dots(act, p, q, pq))) return rc;
        std::vector<int> nxt;
        for (int c : act) {
            if (!(pq[c] > 0.0)) {
                st_[c] = 2;
                continue;
            }
            const double a = rz[c] / pq[c];
            const int64_t N = N_of(hs[c]->g);
            launch_lincomb(x[c], 1.0, x[c], a, p[c], N, st);
            launch_lincomb(r[c], 1.0, r[c], -a, q[c], N, st);
            g_launches += 2;
            nxt.push_back(c);
        }
        act = nxt;
        if ((rc = dots(act, r, r, rr))) return rc;
        nxt.clear();
        for (int c : act) {
            ++it[c];
            rel[c] = std::sqrt(rr[c] / rr0[c]);
            if (rel[c] <= rtol) st_[c] = 0;
            else nxt.push_back(c);
        }
        act = nxt;
        precondition(act);
        if ((rc = dots(act, r, z, rz1))) return rc;
        for (int c : act) {
            launch_lincomb(p[c], 1.0, z[c], rz1[c] / rz[c], p[c], N_of(hs[c]->g), st);
            rz[c] = rz1[c];
        }
        g_launches += (int)act.size();
    }
    HIPCHECK(hipStreamSynchronize(st));
    HIPCHECK(hipGetLastError());
    for (int c = 0; c < K; ++c) {
        if (iters) iters[c] = it[c];
        if (relres) relres[c] = rel[c];
        if (status) status[c] = st_[c];
    }
    return HELM_OK;
}

int hess_pcg(helm_hess_s* h, const double* b, double* x, double p_alpha, double p_mu, double rtol, int maxit,
             hipStream_t st, int32_t* iters, double* relres, helm_info* info) {
    std::vector<helm_info> infos;
    int32_t it = 0, stc = 1;
    double rel = 0.0;
    int rc = hess_pcg_multi({h}, {b}, {x}, p_alpha, p_mu, rtol, maxit, st, &it, &rel, &stc, &infos);
    if (rc) return rc;
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (info) *info = infos[0];
    if (stc == 2) return fail(HELM_ENOCONV, "p.Hp <= 0: the Hessian is not positive definite along a search direction");
    if (stc != 0) return fail(HELM_ENOCONV, "PCG stopped at relative residual " + std::to_string(rel));
    return HELM_OK;
}

// Upper-level derivatives at the context's model m_FWI (sensors at points,
// data given): tau = A^{-1}(g rho u) for every frequency and source (one
// batched solve), then per sensor and coordinate
//   dpsi/dp_{q,l} = -sum Re[(d_l tau)(p_q) conj(eps) + tau(p_q) conj(dd_l - (d_l u)(p_q))]
// and dpsi/dalpha = m^T (Dx^T Dx + Dz^T Dz) rho.  Synchronises the stream.
int hess_upper(helm_hess_s* h, const double* rho, const double* dd, hipStream_t st, double* dp_host,
               double* da_host, helm_info* info) {
    if (!h->full || !h->at_points)
        return fail(HELM_EINVAL, "upper-level derivatives need a context with data and sensors at points");
    if (!rho || !dd || !dp_host || !da_host) return fail(HELM_EINVAL, "bad upper_grad arguments");
    const int64_t N = N_of(h->g);
    const int S = h->S, nw = h->n_omega, Nr = h->Nr;
    const size_t fb = sizeof(double) * 2 * (size_t)N * S;
    Scratch sc(st);
    std::vector<double*> B(nw), T(nw);
    double *dp, *Rrho, *part, *da;
    int rc;
    for (int w = 0; w < nw; ++w) {
        if ((rc = sc.get(&B[w], fb))) return rc;
        if ((rc = sc.get(&T[w], fb))) return rc;
        launch_gn_rhs(coef_of(h->F[w]), h->U[w], N, S, rho, 1, B[w], N, st);
    }
    g_launches += nw;
    std::vector<SolveJob> jobs;
    std::vector<helm_info> infos(nw);
    for (int w = 0; w < nw; ++w) jobs.push_back({h->F[w], B[w], T[w], S, N, &infos[w]});
    if ((rc = solve_jobs(jobs, false, h->tol, st))) return rc;
    if ((rc = sc.get(&dp, sizeof(double) * 2 * Nr))) return rc;
    launch_zero(dp, sizeof(double) * 2 * Nr, st);
    const size_t plane = (size_t)Nr * RTAP;
    for (int w = 0; w < nw; ++w)
        launch_upper(T[w], h->U[w], N, S, h->eps + 2 * (size_t)w * S * Nr, dd + 4 * (size_t)w * S * Nr, h->rnode,
                     h->rw, h->rw + plane, h->rw + 2 * plane, Nr, dp, st);
    const int nblk = (int)((N + 255) / 256);
    if ((rc = sc.get(&Rrho, sizeof(double) * N))) return rc;
    if ((rc = sc.get(&part, sizeof(double) * std::max(nblk, dot_blocks(N))))) return rc;
    if ((rc = sc.get(&da, sizeof(double)))) return rc;
    launch_zero(Rrho, sizeof(double) * N, st);
    launch_gamma(rho, h->g.nx, h->g.nz, 1.0, 0.0, Rrho, part, nblk, st);
    launch_dot(h->m, Rrho, N, part, da, st);
    g_launches += 1 + nw + 4;
    HIPCHECK(hipMemcpyAsync(dp_host, dp, sizeof(double) * 2 * Nr, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(da_host, da, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    HIPCHECK(hipGetLastError());
    if (info) {
        helm_info tot{};
        tot.bad_block = tot.bad_row = -1;
        for (auto& i1 : infos) merge_info(&tot, i1);
        *info = tot;
    }
    return HELM_OK;
}

// ------------------------------------------------------------ L-BFGS FWI --

// Lower-level FWI: minimise phi(m) (eq (newphi)) by L-BFGS with a
// strong-Wolfe line search (the optimiser of App. "Optimisation", after
// Nocedal & Wright): two-loop recursion with initial matrix (s.y / y.y) I;
// the first step along -g scaled to change m by first_change * max|m|;
// trial steps 1, 2, 4, .. until the strong Wolfe conditions hold or a
// bracket is found, then zoom by the safeguarded cubic interpolation
// (bisection when it falls within a tenth of the bracket's ends).  A trial
// model with m_k <= 0 counts as phi = +inf.  All vectors live on the device;
// each evaluation is one hess_build (factor, u, lambda, phi, grad).
struct Fwi {
    const helm_grid* grid;
    int n_omega;
    const double* omegas;
    const double* dobs;
    int S;
    const int32_t* src;
    const double* src_xz;
    int Nr;
    const int32_t* rec;
    const double* rec_xz;
    double alpha, mu;
    int precision;
    double tol;
    hipStream_t st;
    int64_t N;
    double *part, *scal;
    int evals = 0;
    helm_info tot{};

    int dot(const double* a, const double* b, double* out) {
        launch_dot(a, b, N, part, scal, st);
        g_launches += 2;
        HIPCHECK(hipMemcpyAsync(out, scal, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        return HELM_OK;
    }
    int absmax(const double* a, double* out) {
        const int nb = dot_blocks(N);
        std::vector<double> h(nb);
        launch_absmax(a, N, part, st);
        g_launches += 1;
        HIPCHECK(hipMemcpyAsync(h.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        double mx = 0.0;
        for (double v : h) mx = std::max(mx, v);
        *out = mx;
        return HELM_OK;
    }
    // phi and grad at x; *f = +inf (grad untouched) where some m_k <= 0
    int eval(const double* x, double* f, double* g) {
        ++evals;
        int rc = check_model(x, N, st);
        if (rc == HELM_EINVAL) {
            *f = INFINITY;
            return HELM_OK;
        }
        if (rc) return rc;
        helm_hess_s* h = nullptr;
        helm_info inf{};
        rc = hess_build(grid, x, n_omega, omegas, dobs, S, src, src_xz, Nr, rec, rec_xz, alpha, mu, precision, tol,
                        st, f, g, &inf, &h);
        hess_free(h);
        if (rc) return rc;
        merge_info(&tot, inf);
        return HELM_OK;
    }
};

int fwi_run(Fwi& P, double* x, const helm_lbfgs_opts& o, double* hist, helm_fwi_info* out) {
    const int64_t N = P.N;
    const size_t vb = sizeof(double) * N;
    const int mem = o.memory;
    hipStream_t st = P.st;
    Scratch sc(st);
    double *g, *p, *xt, *gt, *q;
    // mem + 1 slots: the pairs in use plus one for the step being taken
    std::vector<double*> Sv(mem + 1), Yv(mem + 1);
    int rc;
    for (double** b : {&g, &p, &xt, &gt, &q})
        if ((rc = sc.get(b, vb))) return rc;
    for (int i = 0; i <= mem; ++i) {
        if ((rc = sc.get(&Sv[i], vb))) return rc;
        if ((rc = sc.get(&Yv[i], vb))) return rc;
    }
    if ((rc = sc.get(&P.part, sizeof(double) * dot_blocks(N)))) return rc;
    if ((rc = sc.get(&P.scal, sizeof(double) * 2))) return rc;
    double f = 0.0;
    if ((rc = P.eval(x, &f, g))) return rc;
    if (!std::isfinite(f)) return fail(HELM_EINVAL, "the start model must be positive");
    double gg;
    if ((rc = P.dot(g, g, &gg))) return rc;
    const double gn0 = std::sqrt(gg);
    out->phi0 = f;
    out->gnorm0 = gn0;
    if (hist) hist[0] = f;
    // pairs in use, oldest first (slot indices), and their s.y
    std::vector<int> order;
    std::vector<double> ys(mem + 1, 0.0);
    int status = 1, it = 0;
    for (;;) {
        if (std::sqrt(gg) <= o.gtol * gn0) {
            status = 0;
            break;
        }
        if (it >= o.max_iters) break;
        // two-loop recursion: p = -H g
        launch_lincomb(q, 1.0, g, 0.0, g, N, st);
        g_launches += 1;
        std::vector<double> al(order.size());
        for (int k = (int)order.size() - 1; k >= 0; --k) {
            const int i = order[k];
            double sq;
            if ((rc = P.dot(Sv[i], q, &sq))) return rc;
            al[k] = sq / ys[i];
            launch_lincomb(q, 1.0, q, -al[k], Yv[i], N, st);
            g_launches += 1;
        }
        if (!order.empty()) {
            const int i = order.back();
            double yy;
            if ((rc = P.dot(Yv[i], Yv[i], &yy))) return rc;
            launch_lincomb(q, ys[i] / yy, q, 0.0, q, N, st);
            g_launches += 1;
        }
        for (int k = 0; k < (int)order.size(); ++k) {
            const int i = order[k];
            double yq;
            if ((rc = P.dot(Yv[i], q, &yq))) return rc;
            launch_lincomb(q, 1.0, q, al[k] - yq / ys[i], Sv[i], N, st);
            g_launches += 1;
        }
        launch_lincomb(p, -1.0, q, 0.0, q, N, st);
        g_launches += 1;
        double d0;
        if ((rc = P.dot(g, p, &d0))) return rc;
        double a_try = 1.0;
        if (order.empty() || !(d0 < 0.0)) {
            order.clear();
            launch_lincomb(p, -1.0, g, 0.0, g, N, st);
            g_launches += 1;
            if ((rc = P.dot(g, p, &d0))) return rc;
            double mx, mg;
            if ((rc = P.absmax(x, &mx))) return rc;
            if ((rc = P.absmax(g, &mg))) return rc;
            a_try = o.first_change * mx / mg;
        }
        // trial point: xt = x + a p, its phi, gradient gt and slope gt.p
        auto trial = [&](double a, double* fa, double* da) -> int {
            launch_lincomb(xt, 1.0, x, a, p, N, st);
            g_launches += 1;
            int r = P.eval(xt, fa, gt);
            if (r) return r;
            *da = NAN;
            if (std::isfinite(*fa)) r = P.dot(gt, p, da);
            return r;
        };
        double a_prev = 0.0, f_prev = f, d_prev = d0;
        double lo[3], hi[3];
        bool found = false, bracket = false;
        double a_acc = 0.0, f_acc = 0.0;
        int used = 0;
        for (int i = 0; i < o.max_evals; ++i) {
            double fa, da;
            if ((rc = trial(a_try, &fa, &da))) return rc;
            used = i + 1;
            if (fa > f + o.c1 * a_try * d0 || (i > 0 && fa >= f_prev)) {
                lo[0] = a_prev, lo[1] = f_prev, lo[2] = d_prev;
                hi[0] = a_try, hi[1] = fa, hi[2] = da;
                bracket = true;
                break;
            }
            if (std::fabs(da) <= -o.c2 * d0) {
                found = true;
                a_acc = a_try, f_acc = fa;
                break;
            }
            if (da >= 0.0) {
                lo[0] = a_try, lo[1] = fa, lo[2] = da;
                hi[0] = a_prev, hi[1] = f_prev, hi[2] = d_prev;
                bracket = true;
                break;
            }
            a_prev = a_try, f_prev = fa, d_prev = da;
            a_try *= 2.0;
        }
        if (!found && !bracket) {
            status = 2;
            break;
        }
        int left = o.max_evals - used;
        while (!found && left > 0) {
            const double w = std::fabs(hi[0] - lo[0]);
            double a = NAN;
            bool ok = false;
            if (std::isfinite(hi[1])) {
                // minimiser of the cubic matching f, f' at both ends
                const double d1 = lo[2] + hi[2] - 3.0 * (lo[1] - hi[1]) / (lo[0] - hi[0]);
                const double disc = d1 * d1 - lo[2] * hi[2];
                if (std::isfinite(disc) && disc >= 0.0) {
                    const double d2 = std::copysign(std::sqrt(disc), hi[0] - lo[0]);
                    const double den = hi[2] - lo[2] + 2.0 * d2;
                    if (den != 0.0) {
                        a = hi[0] - (hi[0] - lo[0]) * (hi[2] + d2 - d1) / den;
                        ok = std::min(lo[0], hi[0]) + 0.1 * w <= a && a <= std::max(lo[0], hi[0]) - 0.1 * w;
                    }
                }
            }
            if (!ok) a = 0.5 * (lo[0] + hi[0]);
            double fa, da;
            if ((rc = trial(a, &fa, &da))) return rc;
            --left;
            if (fa > f + o.c1 * a * d0 || fa >= lo[1]) {
                hi[0] = a, hi[1] = fa, hi[2] = da;
            } else {
                if (std::fabs(da) <= -o.c2 * d0) {
                    found = true;
                    a_acc = a, f_acc = fa;
                    break;
                }
                if (da * (hi[0] - lo[0]) >= 0.0) {
                    hi[0] = lo[0], hi[1] = lo[1], hi[2] = lo[2];
                }
                lo[0] = a, lo[1] = fa, lo[2] = da;
            }
        }
        if (!found) {
            status = 2;
            break;
        }
        // accept: s = a p, y = gt - g, x = xt, g = gt
        int slot = 0;
        while (std::find(order.begin(), order.end(), slot) != order.end()) ++slot;
        double* sv = Sv[slot];
        double* yv = Yv[slot];
        launch_lincomb(sv, a_acc, p, 0.0, p, N, st);
        launch_lincomb(yv, 1.0, gt, -1.0, g, N, st);
        launch_lincomb(x, 1.0, x, 1.0, sv, N, st);
        launch_lincomb(g, 1.0, gt, 0.0, gt, N, st);
        g_launches += 4;
        f = f_acc;
        double sy;
        if ((rc = P.dot(sv, yv, &sy))) return rc;
        if (sy > 0.0) {
            if ((int)order.size() == mem) order.erase(order.begin());
            order.push_back(slot);
            ys[slot] = sy;
        }
        ++it;
        if (hist) hist[it] = f;
        if ((rc = P.dot(g, g, &gg))) return rc;
    }
    out->iterations = it;
    out->evals = P.evals;
    out->status = status;
    out->phi = f;
    out->gnorm = std::sqrt(gg);
    HIPCHECK(hipStreamSynchronize(st));
    HIPCHECK(hipGetLastError());
    return HELM_OK;
}

}  // namespace

// ------------------------------------------------------ allocation-free solve --
// The scratch of helm_solve_noalloc: a fixed device array.  Host code never
// passes `scratch` itself (on the host it names a stand-in, not device
// memory); it uses the address hipGetSymbolAddress gives on each device.
constexpr size_t NOALLOC_BYTES = (size_t)256 << 20;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEV] = {};

// device address of the current device's copy of `scratch`, looked up once
// per device
int noalloc_region(void** out) {
    int dev = -1;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) return fail(HELM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(HELM_EDEVICE, "no device address for the fixed scratch region");
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return HELM_OK;
}

// Peak scratch of solve_jobs for one factor and S right-hand sides: the
// sweep buffers (sweep_group) or the residual partials and norms
// (residual_norms*), on top of the complex64 right-hand side and correction
// (complex64 factors) or, when a tolerance is given, the complex128
// residual and correction of an FP64 refinement (complex128 factors).
size_t solve_scratch_bytes(const helm_factor_s* f, int S, double tol) {
    const size_t es = elem_bytes(f->prec), N = (size_t)N_of(f->g), s16 = (size_t)((S + 15) & ~15);
    const size_t sweep = al256(5 * ((size_t)f->np * s16 * es + 256)) + al256(sizeof(SweepTab));
    const size_t nblk = (N + 255) / 256;
    const size_t resid = al256(sizeof(double) * 2 * nblk * S) + al256(sizeof(double) * 2 * S);
    const size_t phase = std::max(sweep, resid);
    if (f->prec == HELM_FP32_IR) return 2 * al256(sizeof(float) * 2 * N * S) + phase;
    if (tol <= 0.0) return sweep;
    return 2 * al256(sizeof(double) * 2 * N * S) + phase;
}
}  // namespace

// ======================================================================= ABI ==
extern "C" {

const char* helm_last_error(void) { return g_err.c_str(); }

int64_t helm_counter(int which) {
    switch (which) {
        case 0: return g_launches.load();
        case 1: return g_solves.load();
        case 4: return (int64_t)g_cache.cached();
        default: return -1;
    }
}

void helm_set_tile_pivoting(int always) { g_force_pivot = always ? 1 : 0; }

size_t helm_set_cache_limit(size_t bytes) { return g_cache.set_limit(bytes); }

void helm_kernel_timing(int enable) {
    g_timer.drain();
    std::lock_guard<std::mutex> lk(g_timer.mu);
    g_timer.enabled = enable;
    for (int k = 0; k < 3; ++k) {
        g_timer.total_ms[k] = 0.0;
        g_timer.count[k] = 0;
    }
}

int helm_kernel_time(int kind, double* total_ms, int64_t* count) {
    if (kind < 0 || kind > 2 || !total_ms || !count) return fail(HELM_EINVAL, "bad kernel kind");
    g_timer.drain();
    std::lock_guard<std::mutex> lk(g_timer.mu);
    *total_ms = g_timer.total_ms[kind];
    *count = g_timer.count[kind];
    return HELM_OK;
}

int helm_factor_bytes(const helm_grid* grid, int precision, size_t* bytes) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!bytes) return fail(HELM_EINVAL, "bytes is NULL");
    if (precision != HELM_FP64 && precision != HELM_FP32_IR) return fail(HELM_EINVAL, "unknown precision");
    *bytes = factor_bytes_of(*grid, precision);
    return HELM_OK;
}

int helm_factor(const helm_grid* grid, const double* m_dev, double omega, int precision, void* stream,
                helm_factor_t* out) {
    if (!grid) return fail(HELM_EINVAL, "grid is NULL");
    const double* ms[1] = {m_dev};
    return factor_many(1, grid, ms, &omega, precision, S_(stream), out);
}

int helm_factor_batch(int32_t count, const helm_grid* grids, const double* const* m_devs, const double* omegas,
                      int precision, void* stream, helm_factor_t* outs) {
    return factor_many(count, grids, m_devs, omegas, precision, S_(stream), outs);
}

void helm_factor_destroy(helm_factor_t f) { destroy(f); }

int helm_solve(helm_factor_t f, const double* B_dev, double* X_dev, int32_t S, int64_t ld, double tol, void* stream,
               helm_info* info) {
    int rc = check_solve_args(f, B_dev, X_dev, S, ld);
    if (rc) return rc;
    std::vector<SolveJob> jobs{{f, B_dev, X_dev, S, ld, info}};
    return solve_jobs(jobs, false, tol, S_(stream));
}

int helm_solve_noalloc(helm_factor_t f, const double* B_dev, double* X_dev, int32_t S, int64_t ld, double tol,
                       void* stream, helm_info* info) {
    int rc = check_solve_args(f, B_dev, X_dev, S, ld);
    if (rc) return rc;
    const size_t need = solve_scratch_bytes(f, S, tol);
    if (need > NOALLOC_BYTES)
        return fail(HELM_EINVAL, "this solve needs " + std::to_string(need) +
                                     " bytes of scratch; the allocation-free limit is " +
                                     std::to_string(NOALLOC_BYTES) + " bytes");
    void* base = nullptr;
    if ((rc = noalloc_region(&base))) return rc;
    Arena arena{(char*)base, NOALLOC_BYTES, 0};
    ArenaScope scope(&arena);
    std::vector<SolveJob> jobs{{f, B_dev, X_dev, S, ld, info}};
    // untracked (tracking would create an event): the caller keeps f alive
    // until work on `stream` that uses it has ended
    return solve_jobs_on(jobs, false, tol, S_(stream));
}

int helm_adjoint_solve(helm_factor_t f, const double* R_dev, double* L_dev, int32_t S, int64_t ld, double tol,
                       void* stream, helm_info* info) {
    int rc = check_solve_args(f, R_dev, L_dev, S, ld);
    if (rc) return rc;
    std::vector<SolveJob> jobs{{f, R_dev, L_dev, S, ld, info}};
    return solve_jobs(jobs, true, tol, S_(stream));
}

int helm_solve_batch(int32_t count, const helm_factor_t* fs, const double* const* B_devs, double* const* X_devs,
                     const int32_t* S, const int64_t* ld, int adjoint, double tol, void* stream, helm_info* infos) {
    if (count <= 0 || !fs || !B_devs || !X_devs || !S || !ld) return fail(HELM_EINVAL, "bad batch arguments");
    std::vector<SolveJob> j64, j32;
    for (int c = 0; c < count; ++c) {
        int rc = check_solve_args(fs[c], B_devs[c], X_devs[c], S[c], ld[c]);
        if (rc) return rc;
        SolveJob jb{fs[c], B_devs[c], X_devs[c], S[c], ld[c], infos ? &infos[c] : nullptr};
        (fs[c]->prec == HELM_FP32_IR ? j32 : j64).push_back(jb);
    }
    int rc = solve_jobs(j64, adjoint != 0, tol, S_(stream));
    if (rc) return rc;
    return solve_jobs(j32, adjoint != 0, tol, S_(stream));
}

int helm_residual(const helm_grid* grid, const double* m_dev, double omega, int adjoint, const double* B_dev,
                  const double* X_dev, double* r_dev, int32_t S, int64_t ld, double* norms_dev, void* stream) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!m_dev || !B_dev || !X_dev || !norms_dev || S <= 0 || ld < N_of(*grid))
        return fail(HELM_EINVAL, "bad residual arguments");
    hipStream_t st = S_(stream);
    Scratch sc(st);
    const int64_t N = N_of(*grid);
    const int nblk = (int)((N + 255) / 256);
    double* partial;
    if ((rc = sc.get(&partial, sizeof(double) * 2 * (size_t)nblk * S))) return rc;
    Coef cf{m_dev, omega, grid->hx, grid->hz, grid->nx, grid->nz};
    // r is written with leading dimension ld when requested
    launch_residual(cf, adjoint, B_dev, ld, X_dev, ld, r_dev, ld, nullptr, S, partial, nblk, st);
    launch_norms_finish(partial, nblk, S, norms_dev, st);
    g_launches += 2;
    HIPCHECK(hipGetLastError());
    return HELM_OK;
}

int helm_misfit_grad(const helm_grid* grid, const double* m_dev, int32_t n_omega, const double* omegas_host,
                     const double* dobs_dev, int32_t S, const int32_t* src_host, int32_t Nr, const int32_t* rec_host,
                     double alpha, double mu, int precision, double tol, void* stream, double* phi_host,
                     double* grad_dev, helm_info* info) {
    if (!dobs_dev || !phi_host || !grad_dev) return fail(HELM_EINVAL, "bad misfit_grad arguments");
    helm_hess_s* h = nullptr;
    int rc = hess_build(grid, m_dev, n_omega, omegas_host, dobs_dev, S, src_host, nullptr, Nr, rec_host, nullptr,
                        alpha, mu, precision, tol, S_(stream), phi_host, grad_dev, info, &h);
    hess_free(h);
    return rc;
}

int helm_gn_hvp(const helm_grid* grid, const double* m_dev, int32_t n_omega, const double* omegas_host, int32_t S,
                const int32_t* src_host, int32_t Nr, const int32_t* rec_host, int32_t n_dir, const double* mt_dev,
                double alpha, double mu, int precision, double tol, void* stream, double* hv_dev, helm_info* info) {
    if (n_dir <= 0 || !mt_dev || !hv_dev) return fail(HELM_EINVAL, "bad gn_hvp arguments");
    helm_hess_s* h = nullptr;
    helm_info i0{};
    int rc = hess_build(grid, m_dev, n_omega, omegas_host, nullptr, S, src_host, nullptr, Nr, rec_host, nullptr,
                        alpha, mu, precision, tol, S_(stream), nullptr, nullptr, &i0, &h);
    if (rc == HELM_OK) rc = hess_apply(h, n_dir, mt_dev, hv_dev, S_(stream), info);
    if (rc == HELM_OK && info) {
        info->solves += i0.solves;
        info->ir_iters = std::max(info->ir_iters, i0.ir_iters);
        info->max_relres = std::max(info->max_relres, i0.max_relres);
    }
    hess_free(h);
    return rc;
}

int helm_hess_create(const helm_grid* grid, const double* m_dev, int32_t n_omega, const double* omegas_host,
                     const double* dobs_dev, int32_t S, const int32_t* src_host, int32_t Nr, const int32_t* rec_host,
                     double alpha, double mu, int precision, double tol, void* stream, double* phi_host,
                     double* grad_dev, helm_info* info, helm_hess_t* out) {
    if (!out) return fail(HELM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dobs_dev && (phi_host || grad_dev)) return fail(HELM_EINVAL, "phi and grad need data");
    helm_hess_s* h = nullptr;
    int rc = hess_build(grid, m_dev, n_omega, omegas_host, dobs_dev, S, src_host, nullptr, Nr, rec_host, nullptr,
                        alpha, mu, precision, tol, S_(stream), phi_host, grad_dev, info, &h);
    if (rc) {
        hess_free(h);
        return rc;
    }
    *out = h;
    return HELM_OK;
}

int helm_hess_create_at(const helm_grid* grid, const double* m_dev, int32_t n_omega, const double* omegas_host,
                        const double* dobs_dev, int32_t S, const int32_t* src_host, const double* src_xz_host,
                        int32_t Nr, const double* rec_xz_host, double alpha, double mu, int precision, double tol,
                        void* stream, double* phi_host, double* grad_dev, helm_info* info, helm_hess_t* out) {
    if (!out) return fail(HELM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!rec_xz_host) return fail(HELM_EINVAL, "sensor position list is NULL");
    if (!dobs_dev && (phi_host || grad_dev)) return fail(HELM_EINVAL, "phi and grad need data");
    helm_hess_s* h = nullptr;
    int rc = hess_build(grid, m_dev, n_omega, omegas_host, dobs_dev, S, src_host, src_xz_host, Nr, nullptr,
                        rec_xz_host, alpha, mu, precision, tol, S_(stream), phi_host, grad_dev, info, &h);
    if (rc) {
        hess_free(h);
        return rc;
    }
    *out = h;
    return HELM_OK;
}

int helm_upper_grad(helm_hess_t h, const double* rho_dev, const double* ddata_dev, void* stream,
                    double* dpsi_dp_host, double* dpsi_dalpha_host, helm_info* info) {
    if (!h) return fail(HELM_EINVAL, "Hessian handle is NULL");
    return hess_upper(h, rho_dev, ddata_dev, S_(stream), dpsi_dp_host, dpsi_dalpha_host, info);
}

int helm_point_sources(const helm_grid* grid, int32_t S, const double* src_xz_host, double* B_dev, int64_t ld,
                       void* stream) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (S <= 0 || !B_dev || ld < N_of(*grid)) return fail(HELM_EINVAL, "bad point_sources arguments");
    if ((rc = check_points(*grid, S, src_xz_host, "source"))) return rc;
    hipStream_t st = S_(stream);
    Scratch sc(st);
    double* dxz;
    if ((rc = sc.get(&dxz, sizeof(double) * 2 * S))) return rc;
    if ((rc = upload_sync(dxz, src_xz_host, sizeof(double) * 2 * S, st))) return rc;
    launch_zero(B_dev, sizeof(double) * 2 * ((size_t)(S - 1) * ld + N_of(*grid)), st);
    launch_point_sources(B_dev, ld, dxz, S, grid->nx, grid->nz, grid->hx, grid->hz, st);
    g_launches += 2;
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st));
    return HELM_OK;
}

int helm_restrict(const helm_grid* grid, int32_t Nr, const double* rec_xz_host, int deriv, const double* U_dev,
                  int32_t S, int64_t ld, double* out_dev, void* stream) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (Nr <= 0 || S <= 0 || !U_dev || !out_dev || deriv < 0 || deriv > 2 || ld < N_of(*grid))
        return fail(HELM_EINVAL, "bad restrict arguments");
    HostRTab rt;
    if ((rc = rtab_points(*grid, Nr, rec_xz_host, &rt))) return rc;
    hipStream_t st = S_(stream);
    Scratch sc(st);
    int* node;
    double* w;
    if ((rc = sc.get(&node, sizeof(int) * rt.node.size()))) return rc;
    if ((rc = sc.get(&w, sizeof(double) * rt.w.size()))) return rc;
    if ((rc = upload_sync(node, rt.node.data(), sizeof(int) * rt.node.size(), st))) return rc;
    if ((rc = upload_sync(w, rt.w.data(), sizeof(double) * rt.w.size(), st))) return rc;
    launch_restrict(U_dev, ld, node, w + (size_t)deriv * Nr * RTAP, RTAP, Nr, S, out_dev, Nr, st);
    g_launches += 1;
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st));
    return HELM_OK;
}

int helm_fwi(const helm_grid* grid, double* m_dev, int32_t n_omega, const double* omegas_host,
             const double* dobs_dev, int32_t S, const int32_t* src_host, const double* src_xz_host, int32_t Nr,
             const int32_t* rec_host, const double* rec_xz_host, double alpha, double mu, int precision, double tol,
             const helm_lbfgs_opts* opts, void* stream, double* phi_hist_host, helm_fwi_info* info) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!m_dev || !dobs_dev || !opts || !info || n_omega <= 0 || S <= 0 || Nr <= 0)
        return fail(HELM_EINVAL, "bad fwi arguments");
    if ((rec_host != nullptr) == (rec_xz_host != nullptr))
        return fail(HELM_EINVAL, "give either receiver nodes or sensor points");
    if ((src_host != nullptr) == (src_xz_host != nullptr))
        return fail(HELM_EINVAL, "give either source nodes or points");
    const helm_lbfgs_opts& o = *opts;
    if (o.memory < 1 || o.max_iters < 0 || o.max_evals < 1 || !(o.gtol >= 0.0) || !(o.c1 > 0.0) ||
        !(o.c1 < o.c2) || !(o.c2 < 1.0) || !(o.first_change > 0.0))
        return fail(HELM_EINVAL, "bad L-BFGS options (need memory >= 1, 0 < c1 < c2 < 1, first_change > 0)");
    Fwi P{grid, n_omega, omegas_host, dobs_dev, S, src_host, src_xz_host, Nr, rec_host, rec_xz_host, alpha, mu,
          precision, tol, S_(stream), N_of(*grid), nullptr, nullptr};
    P.tot.bad_block = P.tot.bad_row = -1;
    *info = helm_fwi_info{};
    rc = fwi_run(P, m_dev, o, phi_hist_host, info);
    info->solves = P.tot.solves;
    return rc;
}

int helm_hess_apply(helm_hess_t h, int32_t n_dir, const double* mt_dev, double* hv_dev, void* stream,
                    helm_info* info) {
    if (!h) return fail(HELM_EINVAL, "Hessian handle is NULL");
    if (n_dir <= 0 || !mt_dev || !hv_dev) return fail(HELM_EINVAL, "bad hess_apply arguments");
    return hess_apply(h, n_dir, mt_dev, hv_dev, S_(stream), info);
}

int helm_hess_pcg(helm_hess_t h, const double* b_dev, double* x_dev, double p_alpha, double p_mu, double rtol,
                  int32_t maxit, void* stream, int32_t* iters, double* relres, helm_info* info) {
    if (!h) return fail(HELM_EINVAL, "Hessian handle is NULL");
    return hess_pcg(h, b_dev, x_dev, p_alpha, p_mu, rtol, maxit, S_(stream), iters, relres, info);
}

int helm_hess_pcg_batch(int32_t count, const helm_hess_t* hs, const double* const* b_devs, double* const* x_devs,
                        double p_alpha, double p_mu, double rtol, int32_t maxit, void* stream, int32_t* iters,
                        double* relres, int32_t* status, helm_info* infos) {
    if (count <= 0 || !hs || !b_devs || !x_devs) return fail(HELM_EINVAL, "bad pcg_batch arguments");
    std::vector<helm_hess_s*> hh(count);
    std::vector<const double*> bb(count);
    std::vector<double*> xx(count);
    for (int c = 0; c < count; ++c) {
        if (!hs[c]) return fail(HELM_EINVAL, "Hessian handle is NULL");
        for (int d = 0; d < c; ++d)
            if (hs[d] == hs[c]) return fail(HELM_EINVAL, "a context appears twice in the batch");
        hh[c] = hs[c];
        bb[c] = b_devs[c];
        xx[c] = x_devs[c];
    }
    std::vector<helm_info> ii;
    int rc = hess_pcg_multi(hh, bb, xx, p_alpha, p_mu, rtol, maxit, S_(stream), iters, relres, status, &ii);
    if (rc == HELM_OK && infos)
        for (int c = 0; c < count; ++c) infos[c] = ii[c];
    return rc;
}

void helm_hess_destroy(helm_hess_t h) { hess_free(h); }

int helm_gamma_solve(const helm_grid* grid, double alpha, double mu, int32_t n, const double* Y_dev, double* X_dev,
                     void* stream) {
    int rc = check_grid(grid);
    if (rc) return rc;
    if (n <= 0 || !Y_dev || !X_dev) return fail(HELM_EINVAL, "bad gamma_solve arguments");
    if (!(mu > 0.0) || !(alpha >= 0.0) || !std::isfinite(alpha) || !std::isfinite(mu))
        return fail(HELM_EINVAL, "Gamma(alpha, mu) needs alpha >= 0 and mu > 0");
    hipStream_t st = S_(stream);
    const int64_t N = N_of(*grid);
    Scratch sc(st);
    double *Cx, *Cz, *eig, *T1, *T2;
    if ((rc = sc.get(&Cx, sizeof(double) * grid->nx * grid->nx))) return rc;
    if ((rc = sc.get(&Cz, sizeof(double) * grid->nz * grid->nz))) return rc;
    if ((rc = sc.get(&eig, sizeof(double) * N))) return rc;
    if ((rc = sc.get(&T1, sizeof(double) * N * n))) return rc;
    if ((rc = sc.get(&T2, sizeof(double) * N * n))) return rc;
    if ((rc = gamma_tables(grid->nx, grid->nz, alpha, mu, Cx, Cz, eig, st))) return rc;
    launch_gamma_solve(Cx, Cz, eig, grid->nx, grid->nz, n, Y_dev, X_dev, T1, T2, st);
    g_launches += 4;
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st));
    return HELM_OK;
}

int helm_tile_inverse(int32_t count, int32_t kb, int pivot, const double* A_dev, double* T_dev, void* stream) {
    if (count <= 0 || (kb != 16 && kb != 32) || !A_dev || !T_dev) return fail(HELM_EINVAL, "bad tile arguments");
    hipStream_t st = S_(stream);
    Scratch sc(st);
    int* status;
    int rc = sc.get(&status, sizeof(int) * count);
    if (rc) return rc;
    launch_zero(status, sizeof(int) * count, st);
    launch_tile_inverse(count, kb, pivot ? 1 : 0, A_dev, T_dev, status, st);
    g_launches += 2;
    std::vector<int> h(count);
    HIPCHECK(hipMemcpyAsync(h.data(), status, sizeof(int) * count, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    for (int c = 0; c < count; ++c) {
        if (h[c] > 0) return fail(HELM_ESINGULAR, "zero pivot in tile " + std::to_string(c));
        if (h[c] < 0) return fail(HELM_ESINGULAR, "pivot below tolerance in tile " + std::to_string(c));
    }
    return HELM_OK;
}

int helm_mfma_probe(int prec, const double* A_dev, const double* B_dev, double* D_dev, void* stream) {
    if ((prec != 0 && prec != 1) || !A_dev || !B_dev || !D_dev) return fail(HELM_EINVAL, "bad probe arguments");
    launch_mfma_probe(prec, A_dev, B_dev, D_dev, S_(stream));
    g_launches += 1;
    HIPCHECK(hipGetLastError());
    return HELM_OK;
}

}  // extern "C"
