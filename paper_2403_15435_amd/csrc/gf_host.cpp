// Host core of the patch library: scenario forests, bathymetry pyramid, patch
// pool, halo descriptors, regrid topology and the C ABI (include/geoflood.h).
#include "../../include/geoflood.h"
#include "gf_internal.h"
#include "gf_net.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_set>
#include <new>
#include <thread>
#include <vector>

using namespace gf;

namespace {

constexpr int kMaxHydro = 16;
constexpr int kMaxGauges = 256;

struct Leaf {
    int32_t level;
    int64_t PI, PJ;   // global patch index at `level`
    int32_t slot;
};

inline uint64_t key_of(int level, int64_t PI, int64_t PJ)
{
    return ((uint64_t)(level + 1) << 56) | ((uint64_t)PI << 28) | (uint64_t)PJ;
}

// Leaf key -> leaf index: open addressing with linear probing, capacity a
// power of two kept at least twice the entries.  Key and value share an
// entry (one cache line per probe), and an entry is live only when it carries
// the current generation, so that clearing the map (once per regrid, for the
// whole leaf list) costs nothing until the generation counter wraps.  The map
// is never iterated: its layout cannot change a result.
class LeafMap {
    struct Entry {
        uint64_t key;
        int32_t val;
        uint32_t gen;
    };
    std::vector<Entry> tab_;
    size_t mask_ = 0, size_ = 0;
    uint32_t gen_ = 1;
    void grow()
    {
        std::vector<Entry> old;
        old.swap(tab_);
        const uint32_t g = gen_;
        reset(2 * size_ + 16);
        for (const Entry &e : old)
            if (e.gen == g) set(e.key, e.val);
    }
    static uint64_t mix(uint64_t k)
    {
        k ^= k >> 33;
        k *= 0xff51afd7ed558ccdull;
        k ^= k >> 33;
        return k;
    }

public:
    void reset(size_t n)
    {
        size_t cap = 16;
        while (cap < 2 * n + 2) cap <<= 1;
        if (cap != tab_.size()) {
            tab_.assign(cap, Entry{0, -1, 0});
            gen_ = 1;
        } else if (++gen_ == 0) {
            std::fill(tab_.begin(), tab_.end(), Entry{0, -1, 0});
            gen_ = 1;
        }
        mask_ = cap - 1;
        size_ = 0;
    }
    void set(uint64_t k, int32_t v)
    {
        if (2 * (size_ + 1) > tab_.size()) grow();
        size_t i = mix(k) & mask_;
        while (tab_[i].gen == gen_ && tab_[i].key != k) i = (i + 1) & mask_;
        Entry &e = tab_[i];
        if (e.gen != gen_) {
            ++size_;
            e.gen = gen_;
            e.key = k;
        }
        e.val = v;
    }
    // insert k (value 1) if absent; true if it was absent
    bool insert(uint64_t k)
    {
        if (get(k) >= 0) return false;
        set(k, 1);
        return true;
    }
    bool contains(uint64_t k) const { return get(k) >= 0; }
    // -1 when absent
    int32_t get(uint64_t k) const
    {
        if (tab_.empty()) return -1;
        for (size_t i = mix(k) & mask_;; i = (i + 1) & mask_) {
            const Entry &e = tab_[i];
            if (e.gen != gen_) return -1;
            if (e.key == k) return e.val;
        }
    }
};

// Allocator of page-locked host memory: the patch descriptors are rebuilt
// and uploaded after every regrid, and uploads from locked memory run at
// full link speed without staging.
template <typename T>
struct PinnedAlloc {
    using value_type = T;
    PinnedAlloc() = default;
    template <typename U>
    PinnedAlloc(const PinnedAlloc<U> &) {}
    T *allocate(size_t n)
    {
        void *p = nullptr;
        if (hipHostMalloc(&p, n * sizeof(T), hipHostMallocDefault) != hipSuccess) throw std::bad_alloc();
        return (T *)p;
    }
    void deallocate(T *p, size_t) { (void)hipHostFree(p); }
    template <typename U>
    bool operator==(const PinnedAlloc<U> &) const { return true; }
    template <typename U>
    bool operator!=(const PinnedAlloc<U> &) const { return false; }
};

// bits of x (up to 32) spread to the even bit positions
inline uint64_t spread_bits(uint64_t x)
{
    x &= 0xFFFFFFFFull;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// Morton code: x in the even bits, y in the odd bits
inline uint64_t interleave(uint64_t x, uint64_t y) { return spread_bits(x) | (spread_bits(y) << 1); }

struct Scen {
    gf_scenario_desc d{};
    std::vector<double> hydro;
    int dem_level = -1;
    int64_t dem_nx = 0, dem_ny = 0;
    std::vector<double> dem;
    std::vector<std::vector<double>> pyr;   // levels 0..dem_level
    std::vector<Leaf> leaves;
    LeafMap map;                            // key -> leaf index
    TagRules rules{};
    double clamp_base = 0.0, bnd_base = 0.0;
};

// a leaf of the list a regrid builds: refined (kind 0, quadrant q of leaf
// src), coarsened into its parent (1, first child src), or kept (2, src)
struct RgPending {
    int kind;
    int64_t src;
    int q;
};

}  // namespace

// Host worker threads kept for the life of a context: a job runs as
// fn(0..n-1), part 0 on the calling thread, and run() returns when every part
// has finished.  Starting threads for each descriptor rebuild (one per
// regrid) cost more than the rebuild itself.
struct WorkerPool {
    explicit WorkerPool(int n) : n_(n)
    {
        for (int t = 1; t < n_; ++t) th_.emplace_back([this, t] { loop(t); });
    }
    ~WorkerPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    int size() const { return n_; }
    void run(const std::function<void(int)> &fn)
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &fn;
            pending_ = n_ - 1;
            ++gen_;
        }
        cv_.notify_all();
        fn(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [this] { return pending_ == 0; });
        job_ = nullptr;
    }

private:
    void loop(int t)
    {
        unsigned seen = 0;
        for (;;) {
            const std::function<void(int)> *job;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                job = job_;
            }
            (*job)(t);
            std::lock_guard<std::mutex> lk(mu_);
            if (--pending_ == 0) done_.notify_one();
        }
    }
    int n_;
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)> *job_ = nullptr;
    unsigned gen_ = 0;
    int pending_ = 0;
    bool stop_ = false;
};

struct gf_ctx {
    gf_config cfg{};
    std::unique_ptr<WorkerPool> pool;   // descriptor rebuilds, started on first use
    int prec = GF_FP64;
    int m = 32;
    int step_threads = 256;   // workgroup size of the step kernel
    int sched_wg = -1;        // step workgroups: 0 one per patch, > 0 that many persistent, -1 the resident count
    int step_pad = 0;         // LDS words of padding per tile row of the step kernel
    int resident[3][2] = {{0, 0}, {0, 0}, {0, 0}};  // resident workgroups per (threads, padding) (cached)
    struct Trial { int32_t nt, sched, pad; double us; };
    std::vector<Trial> tune_trials;  // the last gf_autotune's timings
    uint8_t *dry[2] = {nullptr, nullptr};   // per slot and buffer: all interior cells dry
    uint8_t *d_dstab = nullptr;              // per slot: dry-update state (unknown / last read buffer / stable)
    unsigned long long *d_stats = nullptr;   // patches through the step kernel, stable dry patches
    int32_t *d_wet = nullptr;                // wet work items of the current step
    unsigned *d_wet_count = nullptr;
    unsigned *d_queue = nullptr;
    // plain path: work items grouped by (scenario, level), per-item Courant
    // data, per-scenario ranges and results
    int32_t *d_pitems = nullptr, *d_pnan = nullptr, *d_prange = nullptr;
    double *d_pmax = nullptr, *d_pres = nullptr;
    // bathymetry of new leaves, staged for one upload and a scatter kernel
    void *d_bstage = nullptr;
    int32_t *d_bslots = nullptr;
    int64_t bstage_cap = 0;   // leaves
    // state transfers: packed staging (bytes) and the slot list
    void *d_sstage = nullptr;
    size_t sstage_bytes = 0;
    int32_t *d_sslots = nullptr;
    int64_t sslots_cap = 0;
    bool flags_dirty = true;  // state changed from the host: recompute the dry flags
    size_t es = 8;
    hipStream_t stream = nullptr;
    std::vector<Scen> sc;
    int64_t cap = 0;
    std::vector<int32_t> free_slots;
    // device memory
    void *q[2] = {nullptr, nullptr};
    void *b = nullptr, *bg = nullptr, *reg = nullptr, *ghost = nullptr;
    double *cacc[2] = {nullptr, nullptr}, *bacc[2] = {nullptr, nullptr};
    PatchDesc *d_desc = nullptr;
    PatchDesc *d_fdesc = nullptr;   // descriptors whose dry flags a regrid refreshes
    int64_t fdesc_cap = 0;
    int64_t desc_cap = 0;
    RefluxTask *d_reflux = nullptr;
    int64_t reflux_cap = 0;
    ScenDev *d_scen = nullptr;
    unsigned *d_counter = nullptr;
    int8_t *d_flags = nullptr;
    double *d_mass = nullptr;
    TagRules *d_rules = nullptr;
    void *d_snap = nullptr;          // local time stepping: state at the start of a macro step
    double *d_snap_acc = nullptr;
    int32_t *d_lperm = nullptr;      // patches by level, finest first (one clock span for all scenarios)
    std::vector<int32_t> lts_count;  // patches within d levels of the finest, d = 0, 1, ...
    // gauges: points, their cells on the current mesh, device records
    struct GaugePoint { int32_t scen; double x, y; };
    std::vector<GaugePoint> gauges;
    std::string tune_cache;          // gf_config.autotune_cache, copied
    // this device's copy of the static scratch (gf_mass_static), taken at creation
    double *static_scratch = nullptr;
    hipError_t static_err = hipSuccess;
    GaugeDev *d_gauges = nullptr;
    double *d_grec = nullptr;
    int64_t *d_gcount = nullptr;
    int64_t grec_cap = 0;
    bool gauges_on = true;   // off during the tuner's trial steps
    XferTaskH *d_xfer = nullptr;
    int64_t xfer_cap = 0;
    // host mirrors
    std::vector<PatchDesc, PinnedAlloc<PatchDesc>> desc;
    std::vector<RefluxTask> reflux;
    // descriptor reuse across a regrid: the descriptors and reflux tasks
    // before it, by slot, and the slots it freed.  A leaf that kept its slot
    // and none of whose halo sources was freed has the same descriptor.
    bool reuse = false;
    std::vector<PatchDesc, PinnedAlloc<PatchDesc>> old_desc;
    std::vector<RefluxTask> old_reflux;
    std::vector<int32_t> old_at, old_task_at;
    std::vector<char> freed_mark;
    std::vector<ScenDev> hs;
    std::vector<int8_t, PinnedAlloc<int8_t>> last_flags;
    bool topo_dirty = true;
    // working memory of gf_regrid, the descriptor rebuild and the budget
    // fold, kept between calls: a regrid of a large mesh changes a few leaves,
    // and buffers of the whole leaf list allocated afresh each time cost more
    // in page faults than the work done in them
    std::vector<Leaf> rg_leaves;
    std::vector<RgPending> rg_pend;
    std::vector<char> rg_ref, rg_coa;
    LeafMap rg_internal;
    std::vector<RefluxTask> rb_task;
    std::vector<char> rb_has, rb_rebuilt;
    // after a regrid: the rebuilt descriptors (new leaves, and leaves next to
    // a change); only their dry flags and dry-update states are refreshed
    std::vector<PatchDesc, PinnedAlloc<PatchDesc>> flag_desc;
    std::vector<double, PinnedAlloc<double>> fold_buf;
    // profiling: prof times the steps with an event pair per stretch of
    // launches (ev[0] before its first step, ev[1] before the next
    // synchronisation); prof_stats has the kernels count patches
    bool prof = false, prof_stats = false, prof_open = false;
    std::vector<hipEvent_t> ev;
    int64_t prof_launches = 0;
    double prof_ms = 0.0;
    // prof_kernel: an event pair around every step-kernel launch alone
    bool prof_kernel = false;
    std::vector<hipEvent_t> kev;     // start, stop of pair i at 2i, 2i + 1
    int64_t kev_n = 0;
    std::string err;
    // learned tagger
    struct Net {
        float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
        uint16_t *wb = nullptr;
        int64_t t = 0;
        float *x = nullptr;                 // staged features [rows][FEAT]
        int8_t *y = nullptr;
        float *logits = nullptr, *loss = nullptr, *part = nullptr;
        float *wtot = nullptr;              // class-weight sum of a device batch
        int64_t n_cap = 0;
        float *featf = nullptr;
        uint16_t *featb = nullptr;
        int64_t feat_cap = 0;
        float *img = nullptr;
        size_t img_cap = 0;
        int32_t *map = nullptr;
        size_t map_cap = 0;
        gfnet::FeatLevel *lv = nullptr;     // 16 levels
        int32_t *lij = nullptr;
        int64_t lij_cap = 0;
    } net;
};

namespace {

int fail(gf_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(gf_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(c, x)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail((c), GF_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

inline int64_t NI(const gf_ctx *c, const Scen &s, int l) { return (int64_t)s.d.mi * c->m << l; }
inline int64_t NJ(const gf_ctx *c, const Scen &s, int l) { return (int64_t)s.d.mj * c->m << l; }
inline double DXl(const gf_ctx *c, const Scen &s, int l) { return (s.d.x1 - s.d.x0) / (double)NI(c, s, l); }
inline double DYl(const gf_ctx *c, const Scen &s, int l) { return (s.d.y1 - s.d.y0) / (double)NJ(c, s, l); }
inline int ring_size(int m) { return (m + 4) * (m + 4) - m * m; }

// ---------------------------------------------------------------- bathymetry
// Cell bathymetry at level l, cell (I, J): integral of the bilinear terrain
// interpolant over the cell (Section 6.2).  Four-point means pair diagonal
// corners so that the result is invariant under exchange of the axes.
double bathy(const gf_ctx *c, const Scen &s, int l, int64_t I, int64_t J)
{
    if (l < s.dem_level) return s.pyr[l][(size_t)(J * NI(c, s, l) + I)];
    const int64_t r = (int64_t)1 << (l - s.dem_level);
    const int64_t i0 = I / r, j0 = J / r;
    auto N = [&](int64_t i, int64_t j) { return s.dem[(size_t)(j * s.dem_nx + i)]; };
    const double n00 = N(i0, j0), n10 = N(i0 + 1, j0), n01 = N(i0, j0 + 1), n11 = N(i0 + 1, j0 + 1);
    if (r == 1) return 0.25 * ((n00 + n11) + (n10 + n01));
    const double fx = ((double)(I - i0 * r) + 0.5) / (double)r;
    const double fy = ((double)(J - j0 * r) + 0.5) / (double)r;
    const double w00 = (1.0 - fx) * (1.0 - fy), w11 = fx * fy, w10 = fx * (1.0 - fy), w01 = (1.0 - fx) * fy;
    return (n00 * w00 + n11 * w11) + (n10 * w10 + n01 * w01);
}

void build_pyramid(const gf_ctx *c, Scen &s)
{
    const int L = s.dem_level;
    s.pyr.assign((size_t)L, {});
    for (int l = L - 1; l >= 0; --l) {
        const int64_t ni = NI(c, s, l), nj = NJ(c, s, l);
        std::vector<double> &P = s.pyr[(size_t)l];
        P.resize((size_t)(ni * nj));
        for (int64_t J = 0; J < nj; ++J)
            for (int64_t I = 0; I < ni; ++I) {
                const double a = bathy(c, s, l + 1, 2 * I, 2 * J), d = bathy(c, s, l + 1, 2 * I + 1, 2 * J + 1);
                const double e = bathy(c, s, l + 1, 2 * I + 1, 2 * J), f = bathy(c, s, l + 1, 2 * I, 2 * J + 1);
                P[(size_t)(J * ni + I)] = 0.25 * ((a + d) + (e + f));
            }
    }
}

// (m+4)^2 bathymetry tile of a leaf: interior and ghost cells from the
// pyramid at the leaf's level; outside the domain the physical rules (x rule,
// then y rule): mirror for walls and inflow sides, copy for extrapolation.
void leaf_bathy_tile(const gf_ctx *c, const Scen &s, const Leaf &L, std::vector<double> &t)
{
    const int m = c->m, TW = m + 4;
    const int64_t ni = NI(c, s, L.level), nj = NJ(c, s, L.level);
    t.assign((size_t)TW * TW, 0.0);
    auto T = [&](int i, int j) -> double & { return t[(size_t)((j + 2) * TW + (i + 2))]; };
    for (int j = -2; j < m + 2; ++j)
        for (int i = -2; i < m + 2; ++i) {
            const int64_t I = L.PI * m + i, J = L.PJ * m + j;
            if (I < 0 || I >= ni || J < 0 || J >= nj) continue;
            T(i, j) = bathy(c, s, L.level, I, J);
        }
    for (int j = -2; j < m + 2; ++j)
        for (int i = -2; i < m + 2; ++i) {
            const int64_t I = L.PI * m + i, J = L.PJ * m + j;
            if (I >= 0 && I < ni) continue;
            if (J < 0 || J >= nj) continue;
            const int side = I < 0 ? 0 : 1, bc = s.d.bc[side];
            int si;
            if (bc == GF_BC_EXTRAP) si = side == 0 ? 0 : m - 1;
            else si = side == 0 ? -1 - i : 2 * m - 1 - i;
            T(i, j) = T(si, j);
        }
    for (int j = -2; j < m + 2; ++j)
        for (int i = -2; i < m + 2; ++i) {
            const int64_t J = L.PJ * m + j;
            if (J >= 0 && J < nj) continue;
            const int side = J < 0 ? 2 : 3, bc = s.d.bc[side];
            int sj;
            if (bc == GF_BC_EXTRAP) sj = side == 2 ? 0 : m - 1;
            else sj = side == 2 ? -1 - j : 2 * m - 1 - j;
            T(i, j) = T(i, sj);
        }
}

template <typename R>
void pack_bathy(const gf_ctx *c, const std::vector<double> &t, R *interior, R *ring)
{
    const int m = c->m, TW = m + 4;
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) interior[j * m + i] = (R)t[(size_t)((j + 2) * TW + (i + 2))];
    int r = 0;
    for (int j = -2; j < 0; ++j)
        for (int i = -2; i < m + 2; ++i) ring[r++] = (R)t[(size_t)((j + 2) * TW + (i + 2))];
    for (int j = m; j < m + 2; ++j)
        for (int i = -2; i < m + 2; ++i) ring[r++] = (R)t[(size_t)((j + 2) * TW + (i + 2))];
    const int cols[4] = {-2, -1, m, m + 1};
    for (int cc = 0; cc < 4; ++cc)
        for (int j = 0; j < m; ++j) ring[r++] = (R)t[(size_t)((j + 2) * TW + (cols[cc] + 2))];
}

// element access helpers for the state buffers
inline size_t fstride(const gf_ctx *c) { return (size_t)c->cap * c->m * c->m; }

// Device staging for state transfers of a scenario's leaves: `bytes` of
// staging and the leaves' slots uploaded in leaf order.
int stage_slots(gf_ctx *c, const Scen &s, size_t bytes)
{
    const int64_t n = (int64_t)s.leaves.size();
    if (bytes > c->sstage_bytes) {
        if (c->d_sstage) (void)hipFree(c->d_sstage);
        c->d_sstage = nullptr;
        c->sstage_bytes = 0;
        HIPCHK(c, hipMalloc(&c->d_sstage, bytes));
        c->sstage_bytes = bytes;
    }
    if (n > c->sslots_cap) {
        if (c->d_sslots) (void)hipFree(c->d_sslots);
        c->d_sslots = nullptr;
        c->sslots_cap = 0;
        HIPCHK(c, hipMalloc(&c->d_sslots, sizeof(int32_t) * (size_t)std::max<int64_t>(n, 256)));
        c->sslots_cap = std::max<int64_t>(n, 256);
    }
    std::vector<int32_t> slots((size_t)n);
    for (int64_t k = 0; k < n; ++k) slots[(size_t)k] = s.leaves[(size_t)k].slot;
    if (n) HIPCHK(c, hipMemcpyAsync(c->d_sslots, slots.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

int launch_state(gf_ctx *c, int kind, const void *a, const void *b, int n, void *out)
{
    const int64_t fs = (int64_t)fstride(c);
    const hipError_t e = c->prec == GF_FP32
        ? gf_launch_state_f32(kind, (const float *)a, (const float *)b, c->d_sslots, n, fs, (float *)out, c->m, c->stream)
        : gf_launch_state_f64(kind, (const double *)a, (const double *)b, c->d_sslots, n, fs, (double *)out, c->m, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "state transfer launch: %s", hipGetErrorString(e));
    return GF_OK;
}

// Bathymetry (interior and halo ring) of the given leaves: packed on the host
// leaf after leaf, one upload, then a kernel copies each to its slot.
int upload_bathy(gf_ctx *c, const Scen &s, const std::vector<Leaf *> &leaves)
{
    const int m = c->m, rs = ring_size(m);
    const size_t MM = (size_t)m * m, per = MM + (size_t)rs;
    const int64_t n = (int64_t)leaves.size();
    if (n == 0) return GF_OK;
    if (n > c->bstage_cap) {
        if (c->d_bstage) (void)hipFree(c->d_bstage);
        if (c->d_bslots) (void)hipFree(c->d_bslots);
        c->d_bstage = nullptr;
        c->d_bslots = nullptr;
        c->bstage_cap = 0;
        const int64_t want = std::max<int64_t>(n, 256);
        HIPCHK(c, hipMalloc(&c->d_bstage, (size_t)want * per * c->es));
        HIPCHK(c, hipMalloc(&c->d_bslots, sizeof(int32_t) * (size_t)want));
        c->bstage_cap = want;
    }
    std::vector<char> host((size_t)n * per * c->es);
    std::vector<int32_t> slots((size_t)n);
    std::vector<double> tile;
    for (int64_t j = 0; j < n; ++j) {
        const Leaf &L = *leaves[(size_t)j];
        slots[(size_t)j] = L.slot;
        leaf_bathy_tile(c, s, L, tile);
        char *dst = host.data() + (size_t)j * per * c->es;
        if (c->prec == GF_FP32) pack_bathy<float>(c, tile, (float *)dst, (float *)dst + MM);
        else pack_bathy<double>(c, tile, (double *)dst, (double *)dst + MM);
    }
    HIPCHK(c, hipMemcpyAsync(c->d_bstage, host.data(), host.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_bslots, slots.data(), sizeof(int32_t) * slots.size(), hipMemcpyHostToDevice, c->stream));
    const hipError_t e = c->prec == GF_FP32
        ? gf_launch_bathy_f32((const float *)c->d_bstage, c->d_bslots, (int)n, (float *)c->b, (float *)c->bg, m, c->stream)
        : gf_launch_bathy_f64((const double *)c->d_bstage, c->d_bslots, (int)n, (double *)c->b, (double *)c->bg, m, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "bathymetry launch: %s", hipGetErrorString(e));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

// ---------------------------------------------------------------- forest
// Leaf order: tree (row-major), then Morton order of the leaf's corner at a
// common resolution of 2^20 inside the tree.  A regrid emits children in
// place of their parent in quadrant order (x low bit) and a parent in place of
// its first child, which keeps this order; the sort only runs when the list
// is out of order (leaves set from outside).  in_order: the caller built the
// list in this order (a regrid), and only the key map is rebuilt.
void sort_leaves(const gf_ctx *c, Scen &s, bool in_order = false)
{
    const int mi = s.d.mi;
    const size_t n = s.leaves.size();
    if (in_order) {
        s.map.reset(n);
        for (size_t k = 0; k < n; ++k) s.map.set(key_of(s.leaves[k].level, s.leaves[k].PI, s.leaves[k].PJ), (int32_t)k);
        return;
    }
    // kept between calls (a regrid sorts the whole list each time)
    static thread_local std::vector<std::pair<int64_t, uint64_t>> key;
    key.resize(n);
    for (size_t k = 0; k < n; ++k) {
        const Leaf &a = s.leaves[k];
        key[k].first = (a.PJ >> a.level) * mi + (a.PI >> a.level);
        key[k].second = interleave((uint64_t)(a.PI & ((1ll << a.level) - 1)) << (20 - a.level),
                                   (uint64_t)(a.PJ & ((1ll << a.level) - 1)) << (20 - a.level));
    }
    if (!std::is_sorted(key.begin(), key.end())) {
        std::vector<size_t> idx(n);
        for (size_t k = 0; k < n; ++k) idx[k] = k;
        std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return key[x] < key[y]; });
        std::vector<Leaf> sorted(n);
        for (size_t k = 0; k < n; ++k) sorted[k] = s.leaves[idx[k]];
        s.leaves.swap(sorted);
    }
    s.map.reset(n);
    for (size_t k = 0; k < n; ++k) s.map.set(key_of(s.leaves[k].level, s.leaves[k].PI, s.leaves[k].PJ), (int32_t)k);
    (void)c;
}

// leaf covering cell (l, I, J) of a scenario: rel 0 same, -1 coarser, +1 finer
int cover(const gf_ctx *c, const Scen &s, int l, int64_t I, int64_t J, int &rel)
{
    const int m = c->m;
    int k = s.map.get(key_of(l, I / m, J / m));
    if (k >= 0) { rel = 0; return k; }
    if (l > 0) {
        k = s.map.get(key_of(l - 1, (I >> 1) / m, (J >> 1) / m));
        if (k >= 0) { rel = -1; return k; }
    }
    k = s.map.get(key_of(l + 1, (2 * I) / m, (2 * J) / m));
    if (k >= 0) { rel = 1; return k; }
    return -1;
}

int32_t take_slot(gf_ctx *c)
{
    if (c->free_slots.empty()) return -1;
    int32_t s = c->free_slots.back();
    c->free_slots.pop_back();
    return s;
}

void give_slot(gf_ctx *c, int32_t s) { c->free_slots.push_back(s); }

// Descriptor of one leaf (halo sources, coarse/fine roles) and, when it is
// the coarse side of a coarse/fine face, its reflux task.  Reads the forest
// only.  Returns false with a message on an unbalanced or uncovered mesh.
bool leaf_desc(const gf_ctx *c, int si, const Scen &s, const Leaf &L, PatchDesc &P, RefluxTask &T, bool &has_task,
               char *err, size_t errn)
{
    const int m = c->m;
    P = PatchDesc{};
    P.slot = L.slot; P.scen = si; P.level = L.level;
    P.PI = (int32_t)L.PI; P.PJ = (int32_t)L.PJ;
    const int64_t ni = NI(c, s, L.level), nj = NJ(c, s, L.level);
    P.dx = DXl(c, s, L.level); P.dy = DYl(c, s, L.level);
    P.xlo = s.d.x0 + (double)(L.PI * m) * P.dx;
    P.ylo = s.d.y0 + (double)(L.PJ * m) * P.dy;
    P.phys = (L.PI == 0 ? 1 : 0) | ((L.PI + 1) * m == ni ? 2 : 0) | (L.PJ == 0 ? 4 : 0) | ((L.PJ + 1) * m == nj ? 8 : 0);
    for (int f = 0; f < 4; ++f) { P.bc[f] = s.d.bc[f]; P.cf_face[f] = -1; P.cf_role[f] = 0; }
    for (int r = 0; r < 12; ++r) {
        int i0, j0;
        switch (r) {
        case 0: i0 = -2; j0 = 0; break;
        case 1: i0 = -2; j0 = m / 2; break;
        case 2: i0 = m; j0 = 0; break;
        case 3: i0 = m; j0 = m / 2; break;
        case 4: i0 = 0; j0 = -2; break;
        case 5: i0 = m / 2; j0 = -2; break;
        case 6: i0 = 0; j0 = m; break;
        case 7: i0 = m / 2; j0 = m; break;
        case 8: i0 = -2; j0 = -2; break;
        case 9: i0 = m; j0 = -2; break;
        case 10: i0 = -2; j0 = m; break;
        default: i0 = m; j0 = m; break;
        }
        const int64_t I = L.PI * m + i0, J = L.PJ * m + j0;
        HaloSrc &h = P.src[r];
        if (I < 0 || I >= ni || J < 0 || J >= nj) { h.kind = HK_PHYS; h.slot = -1; h.oi = h.oj = 0; continue; }
        int rel;
        const int k = cover(c, s, L.level, I, J, rel);
        if (k < 0) {
            snprintf(err, errn, "scenario %d: leaf (l%d,%lld,%lld) has an unbalanced or uncovered neighbour", si, L.level,
                     (long long)L.PI, (long long)L.PJ);
            return false;
        }
        const Leaf &S = s.leaves[(size_t)k];
        h.slot = S.slot;
        if (rel == 0) { h.kind = HK_SAME; h.oi = (int32_t)((L.PI - S.PI) * m); h.oj = (int32_t)((L.PJ - S.PJ) * m); }
        else if (rel == -1) { h.kind = HK_COARSE; h.oi = (int32_t)(L.PI * m - 2 * S.PI * m); h.oj = (int32_t)(L.PJ * m - 2 * S.PJ * m); }
        else { h.kind = HK_FINE; h.oi = (int32_t)(2 * L.PI * m - S.PI * m); h.oj = (int32_t)(2 * L.PJ * m - S.PJ * m); }
    }
    for (int f = 0; f < 4; ++f) {
        const HaloSrc &a = P.src[2 * f], &b2 = P.src[2 * f + 1];
        if (a.kind == HK_FINE && b2.kind == HK_FINE) { P.cf_role[f] = 1; P.cf_face[f] = L.slot * 4 + f; }
        else if (a.kind == HK_COARSE) { P.cf_role[f] = 2; P.cf_face[f] = L.slot * 4 + f; }
        else if ((a.kind == HK_FINE) != (b2.kind == HK_FINE)) {
            snprintf(err, errn, "scenario %d: mixed-level face", si);
            return false;
        }
    }
    T = RefluxTask{};
    has_task = false;
    T.slot = L.slot; T.scen = si; T.area = P.dx * P.dy; T.level = L.level; T.pad = 0;
    for (int f = 0; f < 4; ++f) {
        T.reg_c[f] = -1;
        if (P.cf_role[f] != 1) continue;
        has_task = true;
        T.reg_c[f] = L.slot * 4 + f;
        T.reg_f[f][0] = P.src[2 * f].slot * 4 + (f ^ 1);
        T.reg_f[f][1] = P.src[2 * f + 1].slot * 4 + (f ^ 1);
    }
    return true;
}

// work list: PatchDesc per leaf (scenario order, leaf order) and reflux tasks
// in the same order.  Large meshes are described by several host threads,
// each on a contiguous range of leaves.
// The leaf cell holding each gauge point: cell (I, J) = floor((p - origin) /
// spacing) at a level, the last cell for a point on the far edge; the leaf
// is the one whose patch holds that cell at its own level.
int map_gauges(gf_ctx *c)
{
    if (c->gauges.empty()) return GF_OK;
    std::vector<GaugeDev> g(c->gauges.size());
    for (size_t k = 0; k < c->gauges.size(); ++k) {
        const auto &p = c->gauges[k];
        const Scen &s = c->sc[(size_t)p.scen];
        bool found = false;
        for (int l = s.d.max_level; l >= s.d.min_level && !found; --l) {
            int64_t I = (int64_t)std::floor((p.x - s.d.x0) / DXl(c, s, l));
            int64_t J = (int64_t)std::floor((p.y - s.d.y0) / DYl(c, s, l));
            I = std::min<int64_t>(std::max<int64_t>(I, 0), NI(c, s, l) - 1);
            J = std::min<int64_t>(std::max<int64_t>(J, 0), NJ(c, s, l) - 1);
            const int32_t li = s.map.get(key_of(l, I / c->m, J / c->m));
            if (li < 0) continue;
            const Leaf &L = s.leaves[(size_t)li];
            g[k] = GaugeDev{p.scen, L.slot, (int32_t)((J % c->m) * c->m + (I % c->m)), L.level};
            found = true;
        }
        if (!found) return fail(c, GF_E_INVALID, "gauge %zu: no leaf holds the point", k);
    }
    HIPCHK(c, hipMemcpyAsync(c->d_gauges, g.data(), sizeof(GaugeDev) * g.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

int launch_gauges(gf_ctx *c, int lts)
{
    if (c->gauges.empty() || !c->gauges_on) return GF_OK;
    const int n = (int)c->gauges.size();
    hipError_t e = c->prec == GF_FP32
        ? gf_launch_gauge_f32(c->d_gauges, n, c->d_scen, (const float *)c->q[0], (const float *)c->q[1],
                              (const float *)c->b, c->cap, c->m, c->grec_cap, c->d_grec, c->d_gcount, lts, c->stream)
        : gf_launch_gauge_f64(c->d_gauges, n, c->d_scen, (const double *)c->q[0], (const double *)c->q[1],
                              (const double *)c->b, c->cap, c->m, c->grec_cap, c->d_grec, c->d_gcount, lts, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "gauge launch: %s", hipGetErrorString(e));
    return GF_OK;
}

int rebuild_work(gf_ctx *c)
{
    std::vector<std::pair<int, int64_t>> first;   // (scenario, global index of its first leaf)
    int64_t total = 0;
    for (int si = 0; si < (int)c->sc.size(); ++si) {
        first.push_back({si, total});
        total += (int64_t)c->sc[(size_t)si].leaves.size();
    }
    c->desc.resize((size_t)total);
    // a task entry is read only where has is set, which writes it first
    std::vector<RefluxTask> &task = c->rb_task;
    std::vector<char> &has = c->rb_has, &rebuilt = c->rb_rebuilt;
    task.resize((size_t)total);
    has.assign((size_t)total, 0);
    rebuilt.assign((size_t)total, 0);
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nth = (int)std::min<int64_t>(std::min<unsigned>(hw, 16u), std::max<int64_t>(1, total / 2048));
    if (nth > 1 && (!c->pool || c->pool->size() < nth)) c->pool.reset(new WorkerPool(nth));
    std::vector<std::string> errs((size_t)nth);
    std::vector<int64_t> err_at((size_t)nth, -1);
    auto work = [&](int t) {
        const int64_t lo = total * t / nth, hi = total * (t + 1) / nth;
        size_t sp = 0;
        while (sp + 1 < first.size() && first[sp + 1].second <= lo) ++sp;
        char buf[256];
        for (int64_t g = lo; g < hi; ++g) {
            while (sp + 1 < first.size() && first[sp + 1].second <= g) ++sp;
            const int si = first[sp].first;
            const Scen &s = c->sc[(size_t)si];
            const Leaf &L = s.leaves[(size_t)(g - first[sp].second)];
            if (c->reuse) {
                const int32_t o = c->old_at[(size_t)L.slot];
                if (o >= 0) {
                    const PatchDesc &Q = c->old_desc[(size_t)o];
                    bool same = true;
                    for (int r = 0; r < 12 && same; ++r)
                        if (Q.src[r].kind != HK_PHYS && c->freed_mark[(size_t)Q.src[r].slot]) same = false;
                    if (same) {
                        c->desc[(size_t)g] = Q;
                        const int32_t ti = c->old_task_at[(size_t)L.slot];
                        has[(size_t)g] = ti >= 0;
                        if (ti >= 0) task[(size_t)g] = c->old_reflux[(size_t)ti];
                        continue;
                    }
                }
            }
            bool ht = false;
            if (!leaf_desc(c, si, s, L, c->desc[(size_t)g], task[(size_t)g], ht, buf, sizeof buf)) {
                errs[(size_t)t] = buf;
                err_at[(size_t)t] = g;
                return;
            }
            has[(size_t)g] = ht;
            rebuilt[(size_t)g] = 1;
        }
    };
    if (nth == 1) {
        work(0);
    } else {
        // the pool may be wider than this rebuild needs: extra parts idle
        const std::function<void(int)> job = [&](int t) { if (t < nth) work(t); };
        c->pool->run(job);
    }
    for (int t = 0; t < nth; ++t)
        if (err_at[(size_t)t] >= 0) {
            c->desc.clear();
            return fail(c, GF_E_INVALID, "%s", errs[(size_t)t].c_str());
        }
    c->reflux.clear();
    for (int64_t g = 0; g < total; ++g)
        if (has[(size_t)g]) c->reflux.push_back(task[(size_t)g]);
    c->flag_desc.clear();
    if (c->reuse)
        for (int64_t g = 0; g < total; ++g)
            if (rebuilt[(size_t)g]) c->flag_desc.push_back(c->desc[(size_t)g]);
    bool fresh_alloc = false;
    if ((int64_t)c->desc.size() > c->desc_cap) {
        fresh_alloc = true;
        if (c->d_desc) (void)hipFree(c->d_desc);
        if (c->d_flags) (void)hipFree(c->d_flags);
        if (c->d_mass) (void)hipFree(c->d_mass);
        c->desc_cap = std::max<int64_t>((int64_t)c->desc.size(), 1024);
        HIPCHK(c, hipMalloc(&c->d_desc, sizeof(PatchDesc) * (size_t)c->desc_cap));
        HIPCHK(c, hipMalloc(&c->d_flags, (size_t)c->desc_cap));
        HIPCHK(c, hipMalloc(&c->d_mass, sizeof(double) * (size_t)c->desc_cap));
    }
    if ((int64_t)c->reflux.size() > c->reflux_cap) {
        if (c->d_reflux) (void)hipFree(c->d_reflux);
        c->reflux_cap = std::max<int64_t>((int64_t)c->reflux.size(), 256);
        HIPCHK(c, hipMalloc(&c->d_reflux, sizeof(RefluxTask) * (size_t)c->reflux_cap));
    }
    // after a regrid the descriptors before the first one that was rebuilt or
    // changed index are the bytes the device already holds (a regrid inserts
    // and removes leaves at a few places of an ordered list): only the rest
    // is uploaded
    int64_t kept = 0;
    if (c->reuse && !fresh_alloc)
        while (kept < total && !rebuilt[(size_t)kept] && c->old_at[(size_t)c->desc[(size_t)kept].slot] == kept) ++kept;
    if (kept < total)
        HIPCHK(c, hipMemcpyAsync(c->d_desc + kept, c->desc.data() + kept, sizeof(PatchDesc) * (size_t)(total - kept),
                                 hipMemcpyHostToDevice, c->stream));
    if (!c->reflux.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_reflux, c->reflux.data(), sizeof(RefluxTask) * c->reflux.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->topo_dirty = false;
    return map_gauges(c);
}

int push_scen(gf_ctx *c)
{
    HIPCHK(c, hipMemcpyAsync(c->d_scen, c->hs.data(), sizeof(ScenDev) * c->hs.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

// ends an open profiling stretch (the stream has reached ev[1] once it is
// synchronised)
int prof_mark_end(gf_ctx *c)
{
    if (c->prof_open) HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
    return GF_OK;
}

int prof_collect(gf_ctx *c)
{
    if (!c->prof_open) return GF_OK;
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    c->prof_ms += ms;
    c->prof_open = false;
    return GF_OK;
}

int pull_scen(gf_ctx *c)
{
    int rc = prof_mark_end(c);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->hs.data(), c->d_scen, sizeof(ScenDev) * c->hs.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return prof_collect(c);
}

int ensure_work(gf_ctx *c)
{
    if (c->topo_dirty) return rebuild_work(c);
    return GF_OK;
}


float tau32(double tau)
{
    float tf = (float)tau;
    if ((double)tf > tau) tf = std::nextafter(tf, 0.0f);
    return tf;
}

int refresh_dry_flags(gf_ctx *c)
{
    if (!c->flags_dirty) return GF_OK;
    const int n = (int)c->desc.size();
    hipError_t e;
    if (c->prec == GF_FP32)
        e = gf_launch_dryflag_f32(c->d_desc, n, c->d_scen, (const float *)c->q[0], (const float *)c->q[1], c->dry[0],
                                  c->dry[1], c->d_dstab, c->cap, tau32(c->cfg.dry_tol), c->m, c->stream);
    else
        e = gf_launch_dryflag_f64(c->d_desc, n, c->d_scen, (const double *)c->q[0], (const double *)c->q[1], c->dry[0],
                                  c->dry[1], c->d_dstab, c->cap, c->cfg.dry_tol, c->m, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "dry-flag launch: %s", hipGetErrorString(e));
    c->flags_dirty = false;
    return GF_OK;
}

// After a regrid: the dry flags and dry-update states of the patches whose
// descriptor was rebuilt.  A leaf that kept its slot and its descriptor keeps
// its state, its flag and, since reflux registers are numbered by slot, the
// face records its last dry updates wrote; a new leaf (state moved in by the
// transfer) or one next to a change needs them afresh.  The same kernel as
// the full refresh, over a compact copy of those descriptors.
int refresh_dry_flags_rebuilt(gf_ctx *c)
{
    const int64_t n = (int64_t)c->flag_desc.size();
    if (c->flags_dirty || n == 0) return GF_OK;   // a full refresh is due anyway, or nothing changed
    if (n > c->fdesc_cap) {
        if (c->d_fdesc) (void)hipFree(c->d_fdesc);
        c->d_fdesc = nullptr;
        c->fdesc_cap = 0;
        const int64_t want = std::max<int64_t>(n, 256);
        HIPCHK(c, hipMalloc(&c->d_fdesc, sizeof(PatchDesc) * (size_t)want));
        c->fdesc_cap = want;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_fdesc, c->flag_desc.data(), sizeof(PatchDesc) * (size_t)n, hipMemcpyHostToDevice, c->stream));
    hipError_t e;
    if (c->prec == GF_FP32)
        e = gf_launch_dryflag_f32(c->d_fdesc, (int)n, c->d_scen, (const float *)c->q[0], (const float *)c->q[1], c->dry[0],
                                  c->dry[1], c->d_dstab, c->cap, tau32(c->cfg.dry_tol), c->m, c->stream);
    else
        e = gf_launch_dryflag_f64(c->d_fdesc, (int)n, c->d_scen, (const double *)c->q[0], (const double *)c->q[1], c->dry[0],
                                  c->dry[1], c->d_dstab, c->cap, c->cfg.dry_tol, c->m, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "dry-flag launch: %s", hipGetErrorString(e));
    return GF_OK;
}

// Kernel arguments shared by the fused and the plain path.
template <typename T>
void fill_step_args(gf_ctx *c, StepArgs<T> &a, double dt_fixed, int mode, T tau)
{
    a.desc = c->d_desc; a.n_work = (int)c->desc.size(); a.scen = c->d_scen; a.n_scen = (int)c->sc.size();
    a.q0 = (T *)c->q[0]; a.q1 = (T *)c->q[1]; a.b = (const T *)c->b; a.bg = (const T *)c->bg;
    a.clamp_acc0 = c->cacc[0]; a.clamp_acc1 = c->cacc[1]; a.bnd_acc0 = c->bacc[0]; a.bnd_acc1 = c->bacc[1];
    a.reg = (T *)c->reg; a.cap = c->cap; a.dt_fixed = dt_fixed; a.mode = mode;
    a.g = c->cfg.g; a.cfl_desired = c->cfg.cfl_desired; a.cfl_max = c->cfg.cfl_max;
    a.limiter = c->cfg.limiter; a.transverse = c->cfg.transverse;
    a.tau = tau; a.tau64 = c->cfg.dry_tol; a.done_counter = c->d_counter;
    a.queue = c->d_queue; a.persistent = 0; a.dry0 = c->dry[0]; a.dry1 = c->dry[1];
    a.wet_list = c->d_wet; a.wet_count = c->d_wet_count;
    a.dry_count = c->d_wet_count + 8;   // same 64-byte allocation, another 32-byte sector
    a.dstab = c->d_dstab; a.stats = c->prof_stats ? c->d_stats : nullptr;
}

int launch_reflux(gf_ctx *c, int lts = 0, int tick = 0)
{
    if (c->reflux.empty()) return GF_OK;
    RefluxArgsBase r{};
    r.tasks = c->d_reflux; r.n_tasks = (int)c->reflux.size(); r.scen = c->d_scen; r.cap = c->cap; r.tau64 = c->cfg.dry_tol;
    r.dstab = c->d_dstab;
    r.lts = lts; r.tick = tick;
    hipError_t e;
    if (c->prec == GF_FP32)
        e = gf_launch_reflux_f32(r, (float *)c->q[0], (float *)c->q[1], (const float *)c->reg, c->cacc[0], c->cacc[1], c->dry[0], c->dry[1], c->m, c->stream);
    else
        e = gf_launch_reflux_f64(r, (double *)c->q[0], (double *)c->q[1], (const double *)c->reg, c->cacc[0], c->cacc[1], c->dry[0], c->dry[1], c->m, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "reflux launch: %s", hipGetErrorString(e));
    return GF_OK;
}

// start (which 0) or stop (1) event of the step-kernel launch being issued,
// when the step kernel is timed alone
int kernel_event(gf_ctx *c, int mode, int which)
{
    if (!c->prof_kernel || mode != 0) return GF_OK;
    const size_t need = 2 * (size_t)c->kev_n + 2;
    while (c->kev.size() < need) {
        hipEvent_t x;
        HIPCHK(c, hipEventCreate(&x));
        c->kev.push_back(x);
    }
    HIPCHK(c, hipEventRecord(c->kev[2 * (size_t)c->kev_n + (size_t)which], c->stream));
    if (which == 1) c->kev_n++;
    return GF_OK;
}

int launch_step(gf_ctx *c, double dt_fixed, int mode, int lts = 0, int tick = 0, int n_listed = -1)
{
    const int n = (int)c->desc.size();
    hipError_t e;
    {
        int rc = refresh_dry_flags(c);
        if (rc) return rc;
    }
    // workgroups: one per patch, or the resident count taking patches from the queue
    int grid = n;
    if (c->sched_wg != 0) {
        int want = c->sched_wg;
        if (want < 0) {
            const int base = c->m == 16 ? 64 : 256;
            const int ki = c->step_threads == base ? 0 : (c->step_threads == 2 * base ? 1 : 2);
            int &res = c->resident[ki][c->step_pad];
            if (res <= 0)
                res = c->prec == GF_FP32 ? gf_step_resident_f32(c->m, c->step_threads, c->step_pad)
                                         : gf_step_resident_f64(c->m, c->step_threads, c->step_pad);
            want = res;
        }
        if (want > 0 && want < n) grid = want;
    }
    // a profiled stretch of steps opens with an event before its first launch;
    // no packet goes between the kernels of the stretch
    const bool timed = c->prof && mode == 0;
    if (timed && !c->prof_open) {
        while (c->ev.size() < 2) {
            hipEvent_t x;
            HIPCHK(c, hipEventCreate(&x));
            c->ev.push_back(x);
        }
        HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
        c->prof_open = true;
    }
    // dry_kernel (classification and the dry update) then step_kernel on the
    // wet list
    if (c->prec == GF_FP32) {
        StepArgs<float> a{};
        fill_step_args<float>(c, a, dt_fixed, mode, tau32(c->cfg.dry_tol));
        a.persistent = grid < n ? 1 : 0;
        a.lts = lts; a.tick = tick;
        if (n_listed >= 0) a.wet_list = c->d_lperm;
        e = n_listed >= 0 ? hipMemsetD32Async((hipDeviceptr_t)c->d_wet_count, n_listed, 1, c->stream)
                          : gf_launch_dry_f32(a, c->m, c->stream);
        if (e != hipSuccess) return fail(c, GF_E_HIP, "dry launch: %s", hipGetErrorString(e));
        int rc = kernel_event(c, mode, 0);
        if (rc) return rc;
        e = gf_launch_step_f32(a, c->m, c->step_threads, c->step_pad, grid, c->stream);
    } else {
        StepArgs<double> a{};
        fill_step_args<double>(c, a, dt_fixed, mode, c->cfg.dry_tol);
        a.persistent = grid < n ? 1 : 0;
        a.lts = lts; a.tick = tick;
        if (n_listed >= 0) a.wet_list = c->d_lperm;
        e = n_listed >= 0 ? hipMemsetD32Async((hipDeviceptr_t)c->d_wet_count, n_listed, 1, c->stream)
                          : gf_launch_dry_f64(a, c->m, c->stream);
        if (e != hipSuccess) return fail(c, GF_E_HIP, "dry launch: %s", hipGetErrorString(e));
        int rc = kernel_event(c, mode, 0);
        if (rc) return rc;
        e = gf_launch_step_f64(a, c->m, c->step_threads, c->step_pad, grid, c->stream);
    }
    if (e != hipSuccess) return fail(c, GF_E_HIP, "step launch: %s", hipGetErrorString(e));
    {
        int rc = kernel_event(c, mode, 1);
        if (rc) return rc;
    }
    if (timed) c->prof_launches++;
    // level l ends its step at tick k when 2^(L1 - l) divides k + 1, and only
    // levels below the finest have reflux tasks: none end where k + 1 is odd
    if (mode == 0 && lts) return ((tick + 1) & 1) ? GF_OK : launch_reflux(c, 1, tick);
    if (mode == 0) {
        int rc = launch_reflux(c);
        return rc ? rc : launch_gauges(c, 0);
    }
    return GF_OK;
}

int lts_scen(gf_ctx *c, int phase)
{
    hipError_t e = c->prec == GF_FP32 ? gf_launch_lts_scen_f32(c->d_scen, (int)c->sc.size(), phase, c->stream)
                                      : gf_launch_lts_scen_f64(c->d_scen, (int)c->sc.size(), phase, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "time-stepping phase launch: %s", hipGetErrorString(e));
    return GF_OK;
}

int lts_copy(gf_ctx *c, int dir)
{
    const int n = (int)c->desc.size();
    hipError_t e = c->prec == GF_FP32
        ? gf_launch_lts_copy_f32(c->d_desc, n, c->d_scen, (float *)c->q[0], (float *)c->q[1], c->cacc[0], c->cacc[1],
                                 c->bacc[0], c->bacc[1], (float *)c->d_snap, c->d_snap_acc, c->cap, dir, c->m, c->stream)
        : gf_launch_lts_copy_f64(c->d_desc, n, c->d_scen, (double *)c->q[0], (double *)c->q[1], c->cacc[0], c->cacc[1],
                                 c->bacc[0], c->bacc[1], (double *)c->d_snap, c->d_snap_acc, c->cap, dir, c->m, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "snapshot launch: %s", hipGetErrorString(e));
    return GF_OK;
}

// One macro step of local time stepping (reading R40) for every scenario that
// takes part: snapshot, the ticks, undo where it failed, gauges.
int lts_macro(gf_ctx *c, double dt_fixed, int kmax)
{
    int rc = lts_scen(c, 0);
    if (!rc) rc = lts_copy(c, 0);
    for (int k = 0; k < kmax && !rc; ++k) {
        // with one clock span for every scenario, the patches starting a
        // substep at tick k are those within ctz(k) levels of the finest: a
        // prefix of the list by level (all of it at k = 0)
        int n = -1;
        if (!c->lts_count.empty()) {
            const size_t d = k == 0 ? c->lts_count.size() - 1
                                    : std::min<size_t>((size_t)__builtin_ctz((unsigned)k), c->lts_count.size() - 1);
            n = c->lts_count[d];
        }
        rc = launch_step(c, dt_fixed, 0, 1, k, n);
    }
    if (!rc) rc = lts_copy(c, 1);
    if (!rc) rc = lts_scen(c, 1);
    if (!rc) rc = launch_gauges(c, 1);
    return rc;
}

// The plain path's work list: patch indices grouped by (scenario, level), the
// groups, and each scenario's range of the list.
struct PlainGroup {
    int32_t scen, begin, end;
};

int plain_setup(gf_ctx *c, std::vector<PlainGroup> &groups)
{
    const int n = (int)c->desc.size(), ns = (int)c->sc.size();
    if (!c->ghost) {
        const size_t TW = (size_t)c->m + 4;
        HIPCHK(c, hipMalloc(&c->ghost, (size_t)c->cap * 4 * TW * TW * c->es));
    }
    if (!c->d_pitems) {
        HIPCHK(c, hipMalloc(&c->d_pitems, sizeof(int32_t) * (size_t)c->cap));
        HIPCHK(c, hipMalloc(&c->d_pnan, sizeof(int32_t) * (size_t)c->cap));
        HIPCHK(c, hipMalloc(&c->d_pmax, sizeof(double) * (size_t)c->cap));
        HIPCHK(c, hipMalloc(&c->d_prange, sizeof(int32_t) * 2 * (size_t)ns));
        HIPCHK(c, hipMalloc(&c->d_pres, sizeof(double) * 2 * (size_t)ns));
    }
    std::vector<int32_t> items((size_t)n);
    for (int k = 0; k < n; ++k) items[(size_t)k] = k;
    std::stable_sort(items.begin(), items.end(), [&](int32_t x, int32_t y) {
        const PatchDesc &X = c->desc[(size_t)x], &Y = c->desc[(size_t)y];
        return X.scen != Y.scen ? X.scen < Y.scen : X.level < Y.level;
    });
    groups.clear();
    std::vector<int32_t> range(2 * (size_t)ns, 0);
    for (int k = 0; k < n; ++k) {
        const PatchDesc &P = c->desc[(size_t)items[(size_t)k]];
        if (groups.empty() || groups.back().scen != P.scen || c->desc[(size_t)items[(size_t)groups.back().begin]].level != P.level)
            groups.push_back({P.scen, k, k});
        groups.back().end = k + 1;
        if (range[2 * (size_t)P.scen + 1] == 0) range[2 * (size_t)P.scen] = k;
        range[2 * (size_t)P.scen + 1] = k + 1;
    }
    if (n) HIPCHK(c, hipMemcpyAsync(c->d_pitems, items.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_prange, range.data(), sizeof(int32_t) * range.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

int launch_ghost(gf_ctx *c, const int32_t *items, int n)
{
    hipError_t e;
    if (c->prec == GF_FP32) {
        StepArgs<float> a{};
        fill_step_args<float>(c, a, -1.0, 0, tau32(c->cfg.dry_tol));
        e = gf_launch_ghost_f32(a, items, n, (float *)c->ghost, c->m, c->stream);
    } else {
        StepArgs<double> a{};
        fill_step_args<double>(c, a, -1.0, 0, c->cfg.dry_tol);
        e = gf_launch_ghost_f64(a, items, n, (double *)c->ghost, c->m, c->stream);
    }
    if (e != hipSuccess) return fail(c, GF_E_HIP, "ghost launch: %s", hipGetErrorString(e));
    return GF_OK;
}

// One attempt of the plain path: for every active scenario, per level, the
// ghost fill and then the step from the ghosted tiles; the Courant data
// reduced per scenario and read back; the host accepts or rejects and
// chooses the next step length with the same arithmetic as the device
// controller of the fused path; then the reflux of accepted scenarios.
int plain_attempt(gf_ctx *c, const std::vector<PlainGroup> &groups, double dt_fixed, int mode)
{
    const int ns = (int)c->sc.size();
    const bool fixed = dt_fixed >= 0.0;
    std::vector<char> act((size_t)ns);
    for (int s = 0; s < ns; ++s) {
        const ScenDev &D = c->hs[(size_t)s];
        act[(size_t)s] = D.status == 0 && D.steps < D.target && D.t < D.t_end;
    }
    for (const PlainGroup &g : groups) {
        if (!act[(size_t)g.scen]) continue;
        int rc = launch_ghost(c, c->d_pitems + g.begin, g.end - g.begin);
        if (rc) return rc;
    }
    hipError_t e = hipSuccess;
    for (const PlainGroup &g : groups) {
        if (!act[(size_t)g.scen]) continue;
        const int n = g.end - g.begin;
        if (c->prec == GF_FP32) {
            StepArgs<float> a{};
            fill_step_args<float>(c, a, dt_fixed, mode, tau32(c->cfg.dry_tol));
            e = gf_launch_plain_f32(a, c->d_pitems + g.begin, n, (const float *)c->ghost, c->d_pmax + g.begin,
                                    c->d_pnan + g.begin, c->m, c->stream);
        } else {
            StepArgs<double> a{};
            fill_step_args<double>(c, a, dt_fixed, mode, c->cfg.dry_tol);
            e = gf_launch_plain_f64(a, c->d_pitems + g.begin, n, (const double *)c->ghost, c->d_pmax + g.begin,
                                    c->d_pnan + g.begin, c->m, c->stream);
        }
        if (e != hipSuccess) return fail(c, GF_E_HIP, "plain step launch: %s", hipGetErrorString(e));
    }
    e = c->prec == GF_FP32 ? gf_launch_cflred_f32(c->d_pmax, c->d_pnan, c->d_prange, ns, c->d_pres, c->stream)
                           : gf_launch_cflred_f64(c->d_pmax, c->d_pnan, c->d_prange, ns, c->d_pres, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "Courant reduction launch: %s", hipGetErrorString(e));
    std::vector<double> res(2 * (size_t)ns);
    HIPCHK(c, hipMemcpyAsync(res.data(), c->d_pres, sizeof(double) * res.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool any_accepted = false;
    for (int s = 0; s < ns; ++s) {
        ScenDev &D = c->hs[(size_t)s];
        D.accepted_last = 0;
        if (!act[(size_t)s]) continue;
        const double sm = res[2 * (size_t)s];
        if (mode == 1) {
            D.dt = sm > 0.0 ? c->cfg.cfl_desired / sm : 1.0;
            continue;
        }
        double dtu = fixed ? dt_fixed : D.dt;
        if (!fixed && D.t + dtu > D.t_end) dtu = D.t_end - D.t;
        const double nu = dtu * sm;
        D.dt_used = dtu;
        D.nu_last = nu;
        if (res[2 * (size_t)s + 1] != 0.0) { D.status = -6; continue; }
        if (nu > c->cfg.cfl_max) {
            if (fixed) { D.status = -5; continue; }
            D.rejected += 1;
            D.dt = dtu * c->cfg.cfl_desired / nu;
            continue;
        }
        D.t = D.t + dtu;
        D.steps += 1;
        D.cur ^= 1;
        D.accepted_last = 1;
        D.nu_max = std::max(D.nu_max, nu);
        any_accepted = true;
        if (!fixed) D.dt = nu > 0.0 ? dtu * c->cfg.cfl_desired / nu : dtu;
    }
    int rc = push_scen(c);
    if (rc) return rc;
    if (mode == 0 && any_accepted) {
        rc = launch_reflux(c);
        return rc ? rc : launch_gauges(c, 0);
    }
    return GF_OK;
}

bool scen_ready(const Scen &s) { return s.dem_level >= 0 && !s.leaves.empty(); }

// fold the per-slot clamp/boundary accumulators of the current buffer into
// the scenario totals (leaf order) and clear them
// The fold of the per-slot budget accumulators into each scenario's base, in
// two halves so that a regrid can do its topology work while the copies run:
// fold_begin queues the device-to-host copies; fold_finish waits for them,
// adds the current leaves' values (before the leaf list changes) and queues
// the clears (later device work is ordered after them on the stream).  Until
// fold_finish the device values are untouched, so an error in between loses
// nothing.
int fold_begin(gf_ctx *c)
{
    const size_t cap = (size_t)c->cap;
    c->fold_buf.resize(4 * cap);
    double *ca = c->fold_buf.data(), *cb = ca + cap, *ba = cb + cap, *bb = ba + cap;
    HIPCHK(c, hipMemcpyAsync(ca, c->cacc[0], sizeof(double) * cap, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(cb, c->cacc[1], sizeof(double) * cap, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ba, c->bacc[0], sizeof(double) * cap, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(bb, c->bacc[1], sizeof(double) * cap, hipMemcpyDeviceToHost, c->stream));
    return GF_OK;
}

int fold_finish(gf_ctx *c)
{
    const size_t cap = (size_t)c->cap;
    const double *ca = c->fold_buf.data(), *cb = ca + cap, *ba = cb + cap, *bb = ba + cap;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t si = 0; si < c->sc.size(); ++si) {
        Scen &s = c->sc[si];
        const int cur = c->hs[si].cur;
        for (const Leaf &L : s.leaves) {
            s.clamp_base += cur ? cb[(size_t)L.slot] : ca[(size_t)L.slot];
            s.bnd_base += cur ? bb[(size_t)L.slot] : ba[(size_t)L.slot];
        }
    }
    for (int k = 0; k < 2; ++k) {
        HIPCHK(c, hipMemsetAsync(c->cacc[k], 0, sizeof(double) * cap, c->stream));
        HIPCHK(c, hipMemsetAsync(c->bacc[k], 0, sizeof(double) * cap, c->stream));
    }
    return GF_OK;
}

int fold_accumulators(gf_ctx *c)
{
    const int rc = fold_begin(c);
    return rc ? rc : fold_finish(c);
}

int check_scen(gf_ctx *c, int32_t scen)
{
    if (!c) return GF_E_INVALID;
    if (scen < 0 || scen >= (int32_t)c->sc.size()) return fail(c, GF_E_INVALID, "scenario %d out of range", scen);
    return GF_OK;
}

template <typename R>
void to_real(const double *in, R *out, size_t n) { for (size_t i = 0; i < n; ++i) out[i] = (R)in[i]; }
template <typename R>
void from_real(const R *in, double *out, size_t n) { for (size_t i = 0; i < n; ++i) out[i] = (double)in[i]; }

// device buffer of at least `need` elements (contents not kept)
template <typename T>
hipError_t grow(T **p, int64_t &cap, int64_t need)
{
    if (need <= cap && *p) return hipSuccess;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)std::max<int64_t>(need, 1));
    if (e == hipSuccess) cap = need;
    return e;
}

struct TuneKey {
    std::string text;
};

TuneKey tune_key(const gf_ctx *c)
{
    int64_t n = (int64_t)c->desc.size();
    int64_t bucket = 1;
    while (bucket < n) bucket <<= 1;   // patch count rounded up to a power of two
    char buf[160];
    hipDeviceProp_t prop{};
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    snprintf(buf, sizeof buf, "%s/%s/m%d/n%lld", arch.c_str(), c->prec == GF_FP32 ? "fp32" : "fp64", c->m,
             (long long)bucket);
    return TuneKey{buf};
}

}  // namespace

// =========================================================================
// C ABI
// =========================================================================
extern "C" {

const char *gf_version(void) { return "geoflood-mi355x 0.1"; }

static thread_local char g_create_err[512] = "null context";

const char *gf_last_error(const gf_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_err; }

static bool whole_level(double v) { return v >= 0.0 && v <= 30.0 && v == (double)(int)v; }

// Speed and velocity-depth thresholds non-negative; regions non-empty boxes
// with 0 <= min level <= max level; grades of quantity 0 or 1 with a
// non-negative threshold and a level >= 0.
static bool tag_rules_valid(const gf_scenario_desc &d)
{
    if (!(d.tag_u_refine >= 0.0) || !(d.tag_q_refine >= 0.0)) return false;
    if (d.n_regions < 0 || d.n_regions > kMaxRegions || (d.n_regions > 0 && !d.regions)) return false;
    if (d.n_grades < 0 || d.n_grades > kMaxGrades || (d.n_grades > 0 && !d.grades)) return false;
    for (int r = 0; r < d.n_regions; ++r) {
        const double *v = d.regions + 6 * r;
        if (!(v[2] > v[0]) || !(v[3] > v[1]) || !whole_level(v[4]) || !whole_level(v[5]) || v[5] < v[4]) return false;
    }
    for (int g = 0; g < d.n_grades; ++g) {
        const double *v = d.grades + 3 * g;
        if (!(v[0] == 0.0 || v[0] == 1.0) || !(v[1] >= 0.0) || !whole_level(v[2])) return false;
    }
    return true;
}

static TagRules make_tag_rules(const gf_scenario_desc &d)
{
    TagRules T{};
    T.h = d.tag_h_refine; T.eta = d.tag_eta_refine; T.u = d.tag_u_refine; T.q = d.tag_q_refine;
    T.lmin = d.min_level; T.lmax = d.max_level;
    T.n_regions = d.n_regions; T.n_grades = d.n_grades;
    for (int r = 0; r < d.n_regions; ++r) {
        for (int k = 0; k < 4; ++k) T.region[r][k] = d.regions[6 * r + k];
        T.region_lev[r][0] = (int32_t)d.regions[6 * r + 4];
        T.region_lev[r][1] = (int32_t)d.regions[6 * r + 5];
    }
    for (int g = 0; g < d.n_grades; ++g) {
        T.grade_qty[g] = (int32_t)d.grades[3 * g];
        T.grade_thr[g] = d.grades[3 * g + 1];
        T.grade_lev[g] = (int32_t)d.grades[3 * g + 2];
    }
    return T;
}

int gf_create(const gf_config *cfg, gf_ctx **out)
{
    if (!cfg || !out) return GF_E_INVALID;
    *out = nullptr;
    snprintf(g_create_err, sizeof g_create_err, "invalid configuration");
    if (cfg->m != 16 && cfg->m != 32) return GF_E_UNSUPPORTED;
    if (cfg->precision != GF_FP32 && cfg->precision != GF_FP64) return GF_E_INVALID;
    if (cfg->n_scen <= 0 || !cfg->scen || cfg->max_patches <= 0) return GF_E_INVALID;
    if (!(cfg->g > 0) || !(cfg->dry_tol > 0) || !(cfg->cfl_desired > 0) || !(cfg->cfl_max >= cfg->cfl_desired)) return GF_E_INVALID;
    if (cfg->limiter < GF_LIMITER_MC || cfg->limiter > GF_LIMITER_NONE) return GF_E_INVALID;
    if (cfg->transverse != GF_TRANSVERSE_CORRECTED && cfg->transverse != GF_TRANSVERSE_NONE) return GF_E_INVALID;
    gf_ctx *c = new gf_ctx();
    c->cfg = *cfg;
    c->cfg.scen = nullptr;
    if (cfg->autotune_cache) c->tune_cache = cfg->autotune_cache;
    c->cfg.autotune_cache = nullptr;
    c->prec = cfg->precision;
    c->m = cfg->m;
    c->step_threads = cfg->m == 16 ? 64 : 256;
    c->es = c->prec == GF_FP32 ? 4 : 8;
    c->stream = (hipStream_t)cfg->hip_stream;
    c->cap = cfg->max_patches;
    c->sc.resize((size_t)cfg->n_scen);
    c->hs.assign((size_t)cfg->n_scen, ScenDev{});
    for (int i = 0; i < cfg->n_scen; ++i) {
        const gf_scenario_desc &d = cfg->scen[i];
        if (d.mi <= 0 || d.mj <= 0 || d.min_level < 0 || d.max_level < d.min_level || d.max_level > 14 ||
            !(d.x1 > d.x0) || !(d.y1 > d.y0) || d.n_hydro < 0 || d.n_hydro > kMaxHydro ||
            (d.n_hydro > 0 && !d.hydro) || !tag_rules_valid(d)) {
            delete c;
            return GF_E_INVALID;
        }
        Scen &s = c->sc[(size_t)i];
        s.d = d;
        s.hydro.assign(d.hydro ? d.hydro : nullptr, d.hydro ? d.hydro + 2 * d.n_hydro : nullptr);
        s.d.hydro = nullptr;
        s.rules = make_tag_rules(d);
        s.d.regions = nullptr;
        s.d.grades = nullptr;
        ScenDev &h = c->hs[(size_t)i];
        h.t = 0.0; h.dt = 0.0; h.t_end = d.t_end; h.manning_n = d.manning_n;
        h.inflow_lo = d.inflow_lo; h.inflow_hi = d.inflow_hi; h.inflow_side = d.inflow_side;
        h.x0 = d.x0; h.y0 = d.y0;
        h.n_hydro = d.n_hydro;
        for (int k = 0; k < d.n_hydro; ++k) { h.hydro_t[k] = d.hydro[2 * k]; h.hydro_q[k] = d.hydro[2 * k + 1]; }
    }
    for (int64_t k = c->cap - 1; k >= 0; --k) c->free_slots.push_back((int32_t)k);
    const size_t MM = (size_t)c->m * c->m;
    auto alloc = [&](void **p, size_t bytes) -> bool {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) e = hipMemsetAsync(*p, 0, bytes, c->stream);
        if (e != hipSuccess) {
            snprintf(g_create_err, sizeof g_create_err, "allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
            return false;
        }
        return true;
    };
    bool ok = true;
    ok = ok && alloc(&c->q[0], 3 * MM * c->cap * c->es) && alloc(&c->q[1], 3 * MM * c->cap * c->es);
    ok = ok && alloc(&c->b, MM * c->cap * c->es) && alloc(&c->bg, (size_t)ring_size(c->m) * c->cap * c->es);
    ok = ok && alloc(&c->reg, (size_t)4 * c->cap * c->m * 3 * c->es);
    ok = ok && alloc((void **)&c->cacc[0], sizeof(double) * c->cap) && alloc((void **)&c->cacc[1], sizeof(double) * c->cap);
    ok = ok && alloc((void **)&c->bacc[0], sizeof(double) * c->cap) && alloc((void **)&c->bacc[1], sizeof(double) * c->cap);
    ok = ok && alloc((void **)&c->d_scen, sizeof(ScenDev) * c->sc.size()) && alloc((void **)&c->d_counter, 64 * ((size_t)c->cap / 64 + 2));
    ok = ok && alloc((void **)&c->d_queue, 64) && alloc((void **)&c->dry[0], (size_t)c->cap) &&
         alloc((void **)&c->dry[1], (size_t)c->cap);
    ok = ok && alloc((void **)&c->d_wet, sizeof(int32_t) * (size_t)c->cap) && alloc((void **)&c->d_wet_count, 64);
    ok = ok && alloc((void **)&c->d_dstab, (size_t)c->cap) && alloc((void **)&c->d_stats, 8 * 8 * 65);
    ok = ok && alloc((void **)&c->d_rules, sizeof(TagRules) * c->sc.size());
    if (!ok) {
        gf_destroy(c);
        return GF_E_NOMEM;
    }
    // the static scratch's address on this device, once, with the device current
    c->static_err = gf_static_scratch(&c->static_scratch);
    std::vector<TagRules> rules;
    for (auto &s : c->sc) rules.push_back(s.rules);
    if (hipMemcpyAsync(c->d_rules, rules.data(), sizeof(TagRules) * rules.size(), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        push_scen(c) != GF_OK || hipStreamSynchronize(c->stream) != hipSuccess) {
        gf_destroy(c);
        return GF_E_HIP;
    }
    *out = c;
    return GF_OK;
}

void gf_destroy(gf_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    void *ps[] = {c->q[0], c->q[1], c->b, c->bg, c->reg, c->ghost, c->cacc[0], c->cacc[1], c->bacc[0], c->bacc[1],
                  c->d_desc, c->d_reflux, c->d_scen, c->d_counter, c->d_flags, c->d_rules, c->d_mass, c->d_xfer,
                  c->d_queue, c->dry[0], c->dry[1], c->d_wet, c->d_wet_count, c->d_pitems, c->d_pnan,
                  c->d_prange, c->d_pmax, c->d_pres, c->d_bstage, c->d_bslots, c->d_dstab, c->d_stats,
                  c->d_sstage, c->d_sslots, c->d_gauges, c->d_grec, c->d_gcount, c->d_snap, c->d_snap_acc,
                  c->d_lperm, c->d_fdesc};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    void *pn[] = {c->net.w, c->net.m, c->net.v, c->net.g, c->net.wb, c->net.x, c->net.y, c->net.logits, c->net.loss,
                  c->net.part, c->net.featf, c->net.featb, c->net.img, c->net.map, c->net.lv, c->net.lij,
                  c->net.wtot};
    for (void *p : pn)
        if (p) (void)hipFree(p);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->kev) (void)hipEventDestroy(e);
    delete c;
}

int gf_set_bathymetry(gf_ctx *c, int32_t scen, const double *dem, int64_t nx, int64_t ny, int32_t dem_level)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    Scen &s = c->sc[(size_t)scen];
    if (!dem || dem_level < 0 || dem_level > 14) return fail(c, GF_E_INVALID, "bad terrain arguments");
    if (nx != NI(c, s, dem_level) + 1 || ny != NJ(c, s, dem_level) + 1)
        return fail(c, GF_E_INVALID, "terrain %lldx%lld does not match level %d (%lldx%lld nodes)", (long long)nx,
                    (long long)ny, dem_level, (long long)NI(c, s, dem_level) + 1, (long long)NJ(c, s, dem_level) + 1);
    s.dem_level = dem_level;
    s.dem_nx = nx;
    s.dem_ny = ny;
    s.dem.assign(dem, dem + nx * ny);
    build_pyramid(c, s);
    if (!s.leaves.empty()) {
        std::vector<Leaf *> all;
        for (auto &L : s.leaves) all.push_back(&L);
        return upload_bathy(c, s, all);
    }
    return GF_OK;
}

int gf_set_leaves(gf_ctx *c, int32_t scen, const int32_t *tlxy, int64_t n)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    Scen &s = c->sc[(size_t)scen];
    if (s.dem_level < 0) return fail(c, GF_E_STATE, "set the bathymetry first");
    if (!tlxy || n <= 0) return fail(c, GF_E_INVALID, "no leaves");
    // validate the tiling: area per tree sums to one, no leaf inside another
    std::vector<Leaf> nl((size_t)n);
    std::unordered_set<uint64_t> keys;
    std::vector<double> area((size_t)s.d.mi * s.d.mj, 0.0);
    for (int64_t k = 0; k < n; ++k) {
        const int32_t t = tlxy[4 * k], l = tlxy[4 * k + 1], ix = tlxy[4 * k + 2], iy = tlxy[4 * k + 3];
        if (t < 0 || t >= s.d.mi * s.d.mj || l < s.d.min_level || l > s.d.max_level || ix < 0 || iy < 0 ||
            ix >= (1 << l) || iy >= (1 << l))
            return fail(c, GF_E_INVALID, "leaf %lld out of range", (long long)k);
        Leaf &L = nl[(size_t)k];
        L.level = l;
        L.PI = (int64_t)(t % s.d.mi) * (1ll << l) + ix;
        L.PJ = (int64_t)(t / s.d.mi) * (1ll << l) + iy;
        if (!keys.insert(key_of(l, L.PI, L.PJ)).second) return fail(c, GF_E_INVALID, "duplicate leaf");
        area[(size_t)t] += std::ldexp(1.0, -2 * l);
    }
    for (const Leaf &L : nl)
        for (int a = L.level - 1; a >= 0; --a)
            if (keys.count(key_of(a, L.PI >> (L.level - a), L.PJ >> (L.level - a))))
                return fail(c, GF_E_INVALID, "overlapping leaves");
    for (double a : area)
        if (a != 1.0) return fail(c, GF_E_INVALID, "leaves do not tile every tree");
    if ((int64_t)c->free_slots.size() + (int64_t)s.leaves.size() < n) return fail(c, GF_E_NOMEM, "patch pool too small");
    for (const Leaf &L : s.leaves) give_slot(c, L.slot);
    s.leaves = nl;
    for (Leaf &L : s.leaves) L.slot = take_slot(c);
    sort_leaves(c, s);
    // zero the state of the new slots in both buffers
    rc = stage_slots(c, s, 0);
    if (rc) return rc;
    rc = launch_state(c, 2, nullptr, c->q[1], (int)s.leaves.size(), c->q[0]);
    if (rc) return rc;
    std::vector<Leaf *> all;
    for (auto &L : s.leaves) all.push_back(&L);
    rc = upload_bathy(c, s, all);
    if (rc) return rc;
    c->topo_dirty = true;
    c->flags_dirty = true;
    rc = ensure_work(c);
    if (rc) { c->topo_dirty = true; return rc; }
    s.clamp_base = 0.0;
    s.bnd_base = 0.0;
    return GF_OK;
}

int gf_get_leaves(gf_ctx *c, int32_t scen, int32_t *tlxy, int64_t cap, int64_t *n)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    const Scen &s = c->sc[(size_t)scen];
    if (n) *n = (int64_t)s.leaves.size();
    if (!tlxy) return GF_OK;
    if (cap < (int64_t)s.leaves.size()) return fail(c, GF_E_INVALID, "leaf buffer too small");
    for (size_t k = 0; k < s.leaves.size(); ++k) {
        const Leaf &L = s.leaves[k];
        const int64_t ti = L.PI >> L.level, tj = L.PJ >> L.level;
        tlxy[4 * k] = (int32_t)(tj * s.d.mi + ti);
        tlxy[4 * k + 1] = L.level;
        tlxy[4 * k + 2] = (int32_t)(L.PI - (ti << L.level));
        tlxy[4 * k + 3] = (int32_t)(L.PJ - (tj << L.level));
    }
    return GF_OK;
}

static int patch_io(gf_ctx *c, int32_t scen, int64_t leaf, int32_t field, double *buf, bool write)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    const Scen &s = c->sc[(size_t)scen];
    if (leaf < 0 || leaf >= (int64_t)s.leaves.size()) return fail(c, GF_E_INVALID, "leaf out of range");
    if (field < 0 || field > 3 || (write && field == 3)) return fail(c, GF_E_INVALID, "bad field");
    if (!buf) return GF_E_INVALID;
    const size_t MM = (size_t)c->m * c->m;
    const int slot = s.leaves[(size_t)leaf].slot;
    const int cur = c->hs[(size_t)scen].cur;
    char *dev = field == 3 ? (char *)c->b + (size_t)slot * MM * c->es
                           : (char *)c->q[cur] + ((size_t)field * fstride(c) + (size_t)slot * MM) * c->es;
    std::vector<char> tmp(MM * c->es);
    if (write) {
        if (c->prec == GF_FP32) to_real<float>(buf, (float *)tmp.data(), MM);
        else to_real<double>(buf, (double *)tmp.data(), MM);
        HIPCHK(c, hipMemcpyAsync(dev, tmp.data(), tmp.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        // depth sets the dry flags; a written momentum must also end a stable
        // dry patch's skipped updates (a dry update zeroes it)
        if (field <= 2) c->flags_dirty = true;
    } else {
        HIPCHK(c, hipMemcpyAsync(tmp.data(), dev, tmp.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->prec == GF_FP32) from_real<float>((const float *)tmp.data(), buf, MM);
        else from_real<double>((const double *)tmp.data(), buf, MM);
    }
    return GF_OK;
}

int gf_set_patch(gf_ctx *c, int32_t scen, int64_t leaf, int32_t field, const double *in)
{
    return patch_io(c, scen, leaf, field, const_cast<double *>(in), true);
}

int gf_get_patch(gf_ctx *c, int32_t scen, int64_t leaf, int32_t field, double *out)
{
    return patch_io(c, scen, leaf, field, out, false);
}

int gf_set_state(gf_ctx *c, int32_t scen, const double *in)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    if (!in) return GF_E_INVALID;
    const Scen &s = c->sc[(size_t)scen];
    const size_t MM = (size_t)c->m * c->m;
    const int cur = c->hs[(size_t)scen].cur;
    // convert on the host, one upload in leaf order, scattered to the slots
    const size_t n = s.leaves.size();
    std::vector<char> tmp(n * 3 * MM * c->es);
    if (c->prec == GF_FP32) to_real<float>(in, (float *)tmp.data(), n * 3 * MM);
    else to_real<double>(in, (double *)tmp.data(), n * 3 * MM);
    rc = stage_slots(c, s, tmp.size());
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->d_sstage, tmp.data(), tmp.size(), hipMemcpyHostToDevice, c->stream));
    rc = launch_state(c, 1, c->d_sstage, nullptr, (int)n, c->q[cur]);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->flags_dirty = true;
    return GF_OK;
}

int gf_get_state(gf_ctx *c, int32_t scen, double *out)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    if (!out) return GF_E_INVALID;
    const Scen &s = c->sc[(size_t)scen];
    const size_t MM = (size_t)c->m * c->m;
    const int cur = c->hs[(size_t)scen].cur;
    // gathered on the device in leaf order, one download, widened on the host
    const size_t n = s.leaves.size();
    std::vector<char> tmp(n * 4 * MM * c->es);
    rc = stage_slots(c, s, tmp.size());
    if (rc) return rc;
    rc = launch_state(c, 0, c->q[cur], c->b, (int)n, c->d_sstage);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(tmp.data(), c->d_sstage, tmp.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->prec == GF_FP32) from_real<float>((const float *)tmp.data(), out, n * 4 * MM);
    else from_real<double>((const double *)tmp.data(), out, n * 4 * MM);
    return GF_OK;
}

int gf_fill_ghosts(gf_ctx *c)
{
    if (!c) return GF_E_INVALID;
    for (auto &s : c->sc)
        if (!scen_ready(s)) return fail(c, GF_E_STATE, "scenario without bathymetry or leaves");
    int rc = ensure_work(c);
    if (rc) return rc;
    std::vector<PlainGroup> groups;
    rc = plain_setup(c, groups);
    if (rc) return rc;
    rc = launch_ghost(c, c->d_pitems, (int)c->desc.size());
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

int gf_get_ghosted(gf_ctx *c, int32_t scen, int64_t leaf, int32_t field, double *out)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    if (!c->ghost) return fail(c, GF_E_STATE, "call gf_fill_ghosts first");
    const Scen &s = c->sc[(size_t)scen];
    if (leaf < 0 || leaf >= (int64_t)s.leaves.size() || field < 0 || field > 3 || !out) return GF_E_INVALID;
    const size_t TW2 = ((size_t)c->m + 4) * ((size_t)c->m + 4);
    std::vector<char> tmp(TW2 * c->es);
    const char *dev = (const char *)c->ghost + ((size_t)s.leaves[(size_t)leaf].slot * 4 + (size_t)field) * TW2 * c->es;
    HIPCHK(c, hipMemcpyAsync(tmp.data(), dev, tmp.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->prec == GF_FP32) from_real<float>((const float *)tmp.data(), out, TW2);
    else from_real<double>((const double *)tmp.data(), out, TW2);
    return GF_OK;
}

namespace {
// statistics of a gf_step / gf_step_plain call and its status
int step_result(gf_ctx *c, const std::vector<int64_t> &steps0, const std::vector<int64_t> &rej0, gf_step_stats *out,
                std::chrono::steady_clock::time_point t0, const std::vector<int64_t> *work = nullptr)
{
    int status = GF_OK;
    gf_step_stats st{};
    st.t_min = 1e300; st.t_max = -1e300; st.dt_min = 1e300; st.dt_max = -1e300;
    for (size_t i = 0; i < c->hs.size(); ++i) {
        const ScenDev &h = c->hs[i];
        st.cfl_max = std::max(st.cfl_max, h.nu_max);
        if (h.status != 0 && status == GF_OK) status = h.status;
        st.steps += h.steps - steps0[i];
        st.rejected += h.rejected - rej0[i];
        const int64_t cells = work ? (*work)[i] : (int64_t)c->sc[i].leaves.size() * c->m * c->m;
        st.cell_updates += (h.steps - steps0[i]) * cells;
        st.t_min = std::min(st.t_min, h.t); st.t_max = std::max(st.t_max, h.t);
        st.dt_min = std::min(st.dt_min, h.dt); st.dt_max = std::max(st.dt_max, h.dt);
    }
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (out) *out = st;
    if (status == -5) return fail(c, GF_E_CFL, "a fixed step exceeded the maximum Courant number");
    if (status == -6) return fail(c, GF_E_NUMERIC, "non-finite state produced");
    return status;
}
}  // namespace

int gf_step(gf_ctx *c, int32_t nsteps, const double *dt_fixed, gf_step_stats *out)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!c) return GF_E_INVALID;
    if (nsteps < 0) return fail(c, GF_E_INVALID, "negative step count");
    for (auto &s : c->sc)
        if (!scen_ready(s)) return fail(c, GF_E_STATE, "scenario without bathymetry or leaves");
    int rc = ensure_work(c);
    if (rc) return rc;
    std::vector<int64_t> steps0(c->hs.size()), rej0(c->hs.size());
    for (size_t i = 0; i < c->hs.size(); ++i) {
        ScenDev &h = c->hs[i];
        h.status = 0;
        h.nu_max = 0.0;
        h.target = h.steps + nsteps;
        steps0[i] = h.steps;
        rej0[i] = h.rejected;
    }
    rc = push_scen(c);
    if (rc) return rc;
    if (!dt_fixed) {
        bool need = false;
        for (auto &h : c->hs) need = need || h.dt <= 0.0;
        if (need) {
            rc = launch_step(c, -1.0, 1);
            if (rc) return rc;
        }
    }
    for (int k = 0; k < nsteps; ++k) {
        rc = launch_step(c, dt_fixed ? dt_fixed[k] : -1.0, 0);
        if (rc) return rc;
    }
    rc = pull_scen(c);
    if (rc) return rc;
    if (!dt_fixed) {
        // rejected attempts leave scenarios short of their target: keep going
        for (int round = 0; round < 64; ++round) {
            int64_t missing = 0;
            for (auto &h : c->hs)
                if (h.status == 0 && h.t < h.t_end) missing = std::max<int64_t>(missing, h.target - h.steps);
            if (missing <= 0) break;
            for (int64_t k = 0; k < missing; ++k) {
                rc = launch_step(c, -1.0, 0);
                if (rc) return rc;
            }
            rc = pull_scen(c);
            if (rc) return rc;
        }
    }
    return step_result(c, steps0, rej0, out, t0);
}

int gf_step_plain(gf_ctx *c, int32_t nsteps, const double *dt_fixed, gf_step_stats *out)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!c) return GF_E_INVALID;
    if (nsteps < 0) return fail(c, GF_E_INVALID, "negative step count");
    for (auto &s : c->sc)
        if (!scen_ready(s)) return fail(c, GF_E_STATE, "scenario without bathymetry or leaves");
    int rc = ensure_work(c);
    if (rc) return rc;
    std::vector<PlainGroup> groups;
    rc = plain_setup(c, groups);
    if (rc) return rc;
    std::vector<int64_t> steps0(c->hs.size()), rej0(c->hs.size());
    for (size_t i = 0; i < c->hs.size(); ++i) {
        ScenDev &h = c->hs[i];
        h.status = 0;
        h.nu_max = 0.0;
        h.target = h.steps + nsteps;
        steps0[i] = h.steps;
        rej0[i] = h.rejected;
    }
    rc = push_scen(c);
    if (rc) return rc;
    if (!dt_fixed) {
        bool need = false;
        for (auto &h : c->hs) need = need || h.dt <= 0.0;
        if (need) {
            rc = plain_attempt(c, groups, -1.0, 1);
            if (rc) return rc;
        }
    }
    for (int k = 0; k < nsteps; ++k) {
        rc = plain_attempt(c, groups, dt_fixed ? dt_fixed[k] : -1.0, 0);
        if (rc) return rc;
    }
    if (!dt_fixed) {
        // rejected attempts leave scenarios short of their target: keep going
        for (int round = 0; round < 64; ++round) {
            int64_t missing = 0;
            for (auto &h : c->hs)
                if (h.status == 0 && h.t < h.t_end) missing = std::max<int64_t>(missing, h.target - h.steps);
            if (missing <= 0) break;
            for (int64_t k = 0; k < missing; ++k) {
                rc = plain_attempt(c, groups, -1.0, 0);
                if (rc) return rc;
            }
        }
    }
    return step_result(c, steps0, rej0, out, t0);
}

int gf_step_lts(gf_ctx *c, int32_t nsteps, const double *dt_fixed, gf_step_stats *out)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!c) return GF_E_INVALID;
    if (nsteps < 0) return fail(c, GF_E_INVALID, "negative step count");
    for (auto &s : c->sc)
        if (!scen_ready(s)) return fail(c, GF_E_STATE, "scenario without bathymetry or leaves");
    int rc = ensure_work(c);
    if (rc) return rc;
    if (!c->d_snap) {
        HIPCHK(c, hipMalloc(&c->d_snap, 3 * (size_t)c->m * c->m * (size_t)c->cap * c->es));
        HIPCHK(c, hipMalloc((void **)&c->d_snap_acc, 2 * sizeof(double) * (size_t)c->cap));
    }
    // levels present; every level starts from the common buffer; cell
    // updates per macro step
    int kmax = 1;
    std::vector<int64_t> work(c->sc.size(), 0);
    std::vector<int64_t> steps0(c->hs.size()), rej0(c->hs.size());
    for (size_t i = 0; i < c->sc.size(); ++i) {
        const Scen &s = c->sc[i];
        int L0 = 99, L1 = -1;
        for (const Leaf &L : s.leaves) { L0 = std::min(L0, L.level); L1 = std::max(L1, L.level); }
        ScenDev &h = c->hs[i];
        h.L0 = L0; h.L1 = L1;
        for (int l = 0; l < 16; ++l) { h.lcur[l] = h.cur; h.lcur0[l] = h.cur; }
        h.lts_on = 0; h.lts_fail = 0;
        for (const Leaf &L : s.leaves) work[i] += ((int64_t)c->m * c->m) << (L.level - L0);
        kmax = std::max(kmax, 1 << (L1 - L0));
        h.status = 0;
        h.nu_max = 0.0;
        h.target = h.steps + nsteps;
        steps0[i] = h.steps;
        rej0[i] = h.rejected;
    }
    // the patch list by level, finest first, when every scenario spans the
    // same number of levels (then the ticks agree)
    c->lts_count.clear();
    {
        bool same = true;
        for (size_t i = 1; i < c->hs.size(); ++i)
            same = same && c->hs[i].L1 - c->hs[i].L0 == c->hs[0].L1 - c->hs[0].L0;
        if (same && !c->desc.empty()) {
            const int span = c->hs[0].L1 - c->hs[0].L0;
            std::vector<int32_t> perm;
            perm.reserve(c->desc.size());
            c->lts_count.assign((size_t)span + 1, 0);
            for (int d = 0; d <= span; ++d) {
                for (size_t g = 0; g < c->desc.size(); ++g) {
                    const PatchDesc &P = c->desc[g];
                    if (c->hs[(size_t)P.scen].L1 - P.level == d) perm.push_back((int32_t)g);
                }
                c->lts_count[(size_t)d] = (int32_t)perm.size();
            }
            if (!c->d_lperm) HIPCHK(c, hipMalloc((void **)&c->d_lperm, sizeof(int32_t) * (size_t)c->cap));
            HIPCHK(c, hipMemcpyAsync(c->d_lperm, perm.data(), sizeof(int32_t) * perm.size(), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    rc = push_scen(c);
    if (rc) return rc;
    if (!dt_fixed) {
        bool need = false;
        for (auto &h : c->hs) need = need || h.dt <= 0.0;
        if (need) {
            rc = lts_scen(c, 0);
            if (!rc) rc = launch_step(c, -1.0, 1, 1, 0, c->lts_count.empty() ? -1 : c->lts_count.back());
            if (!rc) rc = lts_scen(c, 1);
            if (rc) return rc;
        }
    }
    for (int k = 0; k < nsteps && !rc; ++k) rc = lts_macro(c, dt_fixed ? dt_fixed[k] : -1.0, kmax);
    if (!rc) rc = pull_scen(c);
    if (!rc && !dt_fixed) {
        // rejected macro steps leave scenarios short of their target: keep going
        for (int round = 0; round < 64 && !rc; ++round) {
            int64_t missing = 0;
            for (auto &h : c->hs)
                if (h.status == 0 && h.t < h.t_end) missing = std::max<int64_t>(missing, h.target - h.steps);
            if (missing <= 0) break;
            for (int64_t k = 0; k < missing && !rc; ++k) rc = lts_macro(c, -1.0, kmax);
            if (!rc) rc = pull_scen(c);
        }
    }
    // every patch back to the scenario's common buffer
    if (!rc) rc = lts_copy(c, 2);
    if (!rc) rc = pull_scen(c);
    c->flags_dirty = true;
    if (rc) return rc;
    return step_result(c, steps0, rej0, out, t0, &work);
}

int gf_tag(gf_ctx *c, int32_t mode, int8_t *flags_out, int64_t cap, int64_t *n)
{
    if (!c) return GF_E_INVALID;
    if (mode == GF_TAG_LEARNED) return gf_net_predict(c, flags_out, cap, n);
    if (mode != GF_TAG_PLAIN) return fail(c, GF_E_INVALID, "unknown tagging mode %d", mode);
    int rc = ensure_work(c);
    if (rc) return rc;
    const int nw = (int)c->desc.size();
    hipError_t e;
    if (c->prec == GF_FP32)
        e = gf_launch_tag_f32(c->d_desc, nw, c->d_scen, (const float *)c->q[0], (const float *)c->q[1], (const float *)c->b,
                              c->cap, c->d_rules, c->cfg.dry_tol, c->d_flags, c->m, c->stream);
    else
        e = gf_launch_tag_f64(c->d_desc, nw, c->d_scen, (const double *)c->q[0], (const double *)c->q[1], (const double *)c->b,
                              c->cap, c->d_rules, c->cfg.dry_tol, c->d_flags, c->m, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "tag launch: %s", hipGetErrorString(e));
    c->last_flags.resize((size_t)nw);
    if (nw) HIPCHK(c, hipMemcpyAsync(c->last_flags.data(), c->d_flags, (size_t)nw, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (n) *n = nw;
    if (flags_out) {
        if (cap < nw) return fail(c, GF_E_INVALID, "flag buffer too small");
        std::memcpy(flags_out, c->last_flags.data(), (size_t)nw);
    }
    return GF_OK;
}

// ------------------------------------------------------------------ regrid
namespace {

// Is the level-(l) cell position (X, Y) (in patch units) an interior node of
// the tree described by `internal`?  Positions outside the domain are not.
struct Topo {
    const gf_ctx *c;
    const Scen *s;
    LeafMap &internal;                        // keys of nodes that have children
    bool inside(int l, int64_t X, int64_t Y) const
    {
        return X >= 0 && Y >= 0 && X < ((int64_t)s->d.mi << l) && Y < ((int64_t)s->d.mj << l);
    }
    void add_ancestors(int l, int64_t X, int64_t Y)
    {
        for (int a = l - 1; a >= 0; --a) {
            const uint64_t k = key_of(a, X >> (l - a), Y >> (l - a));
            if (!internal.insert(k)) break;
        }
    }
    // any leaf finer than level l+1 touching the level-l patch (X, Y)?  That is
    // one of its twelve level-(l+1) neighbours being subdivided.
    bool finer_than_next(int l, int64_t X, int64_t Y) const
    {
        const int64_t x0 = 2 * X, y0 = 2 * Y;
        static const int off[12][2] = {{-1, 0}, {-1, 1}, {2, 0}, {2, 1}, {0, -1}, {1, -1}, {0, 2}, {1, 2},
                                       {-1, -1}, {2, -1}, {-1, 2}, {2, 2}};
        for (auto &o : off) {
            const int64_t xx = x0 + o[0], yy = y0 + o[1];
            if (!inside(l + 1, xx, yy)) continue;
            if (internal.contains(key_of(l + 1, xx, yy))) return true;
        }
        return false;
    }
};

}  // namespace

int gf_regrid(gf_ctx *c, const int8_t *flags_in, int64_t *n_leaves)
{
    if (!c) return GF_E_INVALID;
    int rc = ensure_work(c);
    if (rc) return rc;
    const int64_t nw = (int64_t)c->desc.size();
    const int8_t *flags = flags_in ? flags_in : (c->last_flags.size() == (size_t)nw ? c->last_flags.data() : nullptr);
    if (!flags) return fail(c, GF_E_STATE, "no flags: call gf_tag first");
    // the budget fold's copies run under the topology work below; it is
    // finished before the first leaf list changes
    rc = fold_begin(c);
    if (rc) return rc;
    bool folded = false;
    const int m = c->m;
    std::vector<XferTaskH> xfer;
    std::vector<int32_t> freed;
    int64_t off = 0, total = 0;
    bool changed = false;   // a leaf was refined or coarsened in some scenario
    for (size_t si = 0; si < c->sc.size(); ++si) {
        Scen &s = c->sc[si];
        const int64_t n = (int64_t)s.leaves.size();
        const int8_t *fl = flags + off;
        off += n;
        // a scenario where no flag can take effect keeps its leaves (the
        // common case between fronts): none of the work below is needed
        bool cand = false;
        for (int64_t k = 0; k < n && !cand; ++k) {
            const int lv = s.leaves[(size_t)k].level;
            cand = (fl[k] > 0 && lv < s.d.max_level) || (fl[k] < 0 && lv > s.d.min_level);
        }
        if (!cand) {
            total += n;
            continue;
        }
        std::vector<char> &ref = c->rg_ref, &coa = c->rg_coa;
        ref.assign((size_t)n, 0);
        coa.assign((size_t)n, 0);
        for (int64_t k = 0; k < n; ++k) ref[(size_t)k] = fl[k] > 0 && s.leaves[(size_t)k].level < s.d.max_level;
        // 2:1 face+corner balance closure of the refinement: a leaf must
        // refine when one of the twelve next-finer cells around it has
        // children.  The mesh was balanced before, so only a leaf one level
        // coarser than, and next to, a node that gains children can break
        // the rule; the closure follows a worklist of such nodes.
        Topo T{c, &s, c->rg_internal};
        T.internal.reset((size_t)n);
        struct Node { int l; int64_t X, Y; };
        std::vector<Node> work;
        for (int64_t k = 0; k < n; ++k) {
            const Leaf &L = s.leaves[(size_t)k];
            if (ref[(size_t)k]) {
                T.internal.insert(key_of(L.level, L.PI, L.PJ));
                work.push_back({L.level, L.PI, L.PJ});
            }
            T.add_ancestors(L.level, L.PI, L.PJ);
        }
        while (!work.empty()) {
            const Node N = work.back();
            work.pop_back();
            if (N.l == 0) continue;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    const int64_t xx = N.X + dx, yy = N.Y + dy;
                    if (!T.inside(N.l, xx, yy)) continue;
                    const int kk = s.map.get(key_of(N.l - 1, xx >> 1, yy >> 1));
                    if (kk < 0 || ref[(size_t)kk]) continue;
                    const Leaf &L = s.leaves[(size_t)kk];
                    if (L.level >= s.d.max_level) return fail(c, GF_E_INVALID, "balance needs a level beyond max_level");
                    ref[(size_t)kk] = 1;
                    T.internal.insert(key_of(L.level, L.PI, L.PJ));
                    work.push_back({L.level, L.PI, L.PJ});
                }
        }
        // coarsening of complete families whose parent stays balanced
        for (int64_t k = 0; k < n; ++k) {
            const Leaf &L = s.leaves[(size_t)k];
            if (fl[k] >= 0 || ref[(size_t)k] || L.level <= s.d.min_level || (L.PI & 1) || (L.PJ & 1)) continue;
            int sib[4];
            bool ok = true;
            for (int q = 0; q < 4 && ok; ++q) {
                sib[q] = s.map.get(key_of(L.level, L.PI + (q & 1), L.PJ + (q >> 1)));
                if (sib[q] < 0) { ok = false; break; }
                if (fl[sib[q]] >= 0 || ref[(size_t)sib[q]]) ok = false;
            }
            if (!ok) continue;
            if (T.finer_than_next(L.level - 1, L.PI >> 1, L.PJ >> 1)) continue;
            for (int q = 0; q < 4; ++q) coa[(size_t)sib[q]] = 1;
        }
        bool any = false;
        for (int64_t k = 0; k < n && !any; ++k) any = ref[(size_t)k] || coa[(size_t)k];
        if (!any) {
            total += n;
            continue;
        }
        changed = true;
        // new leaves; slots for children and parents are fresh
        std::vector<Leaf> &nl = c->rg_leaves;
        std::vector<Leaf *> fresh;
        int64_t need = 0;
        for (int64_t k = 0; k < n; ++k) need += ref[(size_t)k] ? 4 : 0;
        nl.clear();
        nl.reserve((size_t)n + (size_t)need);
        for (int64_t k = 0; k < n; ++k) need += (coa[(size_t)k] && !(s.leaves[(size_t)k].PI & 1) && !(s.leaves[(size_t)k].PJ & 1)) ? 1 : 0;
        if (need > (int64_t)c->free_slots.size()) return fail(c, GF_E_NOMEM, "patch pool too small for the regrid");
        std::vector<RgPending> &pend = c->rg_pend;
        pend.clear();
        for (int64_t k = 0; k < n; ++k) {
            const Leaf &L = s.leaves[(size_t)k];
            if (ref[(size_t)k]) {
                for (int q = 0; q < 4; ++q) {
                    Leaf C{L.level + 1, 2 * L.PI + (q & 1), 2 * L.PJ + (q >> 1), take_slot(c)};
                    nl.push_back(C);
                    pend.push_back({0, k, q});
                }
                freed.push_back(L.slot);
            } else if (coa[(size_t)k]) {
                if (!(L.PI & 1) && !(L.PJ & 1)) {
                    Leaf P{L.level - 1, L.PI >> 1, L.PJ >> 1, take_slot(c)};
                    nl.push_back(P);
                    pend.push_back({1, k, 0});
                }
                freed.push_back(L.slot);
            } else {
                nl.push_back(L);
                pend.push_back({2, k, 0});
            }
        }
        const std::vector<Leaf> &old = s.leaves;
        const auto &oldmap = s.map;
        // transfer tasks (read the old slots, write the fresh ones)
        for (size_t j = 0; j < nl.size(); ++j) {
            const RgPending &p = pend[j];
            if (p.kind == 2) continue;
            fresh.push_back(&nl[j]);
            XferTaskH t{};
            t.dst = nl[j].slot;
            t.scen = (int32_t)si;
            if (p.kind == 0) {
                t.kind = 0; t.qx = p.q & 1; t.qy = p.q >> 1; t.src[0] = old[(size_t)p.src].slot;
            } else {
                t.kind = 1;
                const Leaf &L = old[(size_t)p.src];
                for (int q = 0; q < 4; ++q) t.src[q] = old[(size_t)oldmap.get(key_of(L.level, L.PI + (q & 1), L.PJ + (q >> 1)))].slot;
            }
            xfer.push_back(t);
        }
        if (!folded) {
            rc = fold_finish(c);
            if (rc) return rc;
            folded = true;
        }
        rc = upload_bathy(c, s, fresh);
        if (rc) return rc;
        s.leaves.swap(nl);   // the old list's memory serves the next regrid
        sort_leaves(c, s, true);   // emitted in order (see sort_leaves): the map only
        total += (int64_t)s.leaves.size();
    }
    if (!changed) {
        // the same leaves, slots, descriptors, reflux tasks, dry flags and
        // dry-update states
        rc = fold_finish(c);
        if (rc) return rc;
        if (n_leaves) *n_leaves = total;
        return GF_OK;
    }
    if (!xfer.empty()) {
        if ((int64_t)xfer.size() > c->xfer_cap) {
            if (c->d_xfer) (void)hipFree(c->d_xfer);
            c->xfer_cap = std::max<int64_t>((int64_t)xfer.size(), 1024);
            HIPCHK(c, hipMalloc(&c->d_xfer, sizeof(XferTaskH) * (size_t)c->xfer_cap));
        }
        HIPCHK(c, hipMemcpyAsync(c->d_xfer, xfer.data(), sizeof(XferTaskH) * xfer.size(), hipMemcpyHostToDevice, c->stream));
        hipError_t e;
        if (c->prec == GF_FP32)
            e = gf_launch_transfer_f32(c->d_xfer, (int)xfer.size(), c->d_scen, (float *)c->q[0], (float *)c->q[1],
                                       (const float *)c->b, c->cap, c->cfg.dry_tol, m, c->stream);
        else
            e = gf_launch_transfer_f64(c->d_xfer, (int)xfer.size(), c->d_scen, (double *)c->q[0], (double *)c->q[1],
                                       (const double *)c->b, c->cap, c->cfg.dry_tol, m, c->stream);
        if (e != hipSuccess) return fail(c, GF_E_HIP, "transfer launch: %s", hipGetErrorString(e));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    // the descriptors of leaves that kept their slot and their sources carry over
    c->old_at.assign((size_t)c->cap, -1);
    c->old_task_at.assign((size_t)c->cap, -1);
    c->freed_mark.assign((size_t)c->cap, 0);
    for (size_t g = 0; g < c->desc.size(); ++g) c->old_at[(size_t)c->desc[g].slot] = (int32_t)g;
    for (size_t t = 0; t < c->reflux.size(); ++t) c->old_task_at[(size_t)c->reflux[t].slot] = (int32_t)t;
    for (int32_t sl : freed) c->freed_mark[(size_t)sl] = 1;
    std::swap(c->desc, c->old_desc);
    std::swap(c->reflux, c->old_reflux);
    c->reuse = true;
    for (int32_t sl : freed) give_slot(c, sl);
    c->topo_dirty = true;
    rc = ensure_work(c);
    c->reuse = false;
    if (rc) return rc;
    rc = refresh_dry_flags_rebuilt(c);
    if (rc) return rc;
    if (n_leaves) *n_leaves = total;
    return GF_OK;
}

// ---------------------------------------------------------------------------
// learned tagger
// ---------------------------------------------------------------------------
namespace {

int net_ready(gf_ctx *c) { return c->net.w ? GF_OK : fail(c, GF_E_STATE, "network parameters not set"); }

int net_stage_batch(gf_ctx *c, const double *x, int32_t n)
{
    auto &N = c->net;
    if (n > N.n_cap) {
        int64_t cap = N.n_cap;
        int64_t c1 = cap, c2 = cap, c3 = cap, c4 = cap, c5 = cap;
        hipError_t e = grow(&N.x, c1, (int64_t)n * gfnet::FEAT);
        if (e == hipSuccess) e = grow(&N.y, c2, n);
        if (e == hipSuccess) e = grow(&N.logits, c3, (int64_t)n * 3);
        if (e == hipSuccess) e = grow(&N.loss, c4, n);
        if (e == hipSuccess) e = grow(&N.part, c5, (int64_t)n * gfnet::N_PARAMS);
        if (e != hipSuccess) { N.n_cap = 0; return fail(c, GF_E_NOMEM, "network batch buffers: %s", hipGetErrorString(e)); }
        N.n_cap = n;
    }
    if (x) {
        std::vector<float> xf((size_t)n * gfnet::FEAT);
        for (size_t i = 0; i < xf.size(); ++i) xf[i] = (float)x[i];
        HIPCHK(c, hipMemcpyAsync(N.x, xf.data(), sizeof(float) * xf.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return GF_OK;
}

// feature tiles of every leaf of every scenario (leaf order) into featf/featb
int net_features(gf_ctx *c, int64_t *n_out)
{
    auto &N = c->net;
    int rc = ensure_work(c);
    if (rc) return rc;
    rc = pull_scen(c);
    if (rc) return rc;
    int64_t total = 0;
    for (auto &s : c->sc) total += (int64_t)s.leaves.size();
    int64_t cap1 = N.feat_cap, cap2 = N.feat_cap;
    if (total > N.feat_cap) {
        if (grow(&N.featf, cap1, total * gfnet::FEAT) != hipSuccess || grow(&N.featb, cap2, total * gfnet::FEAT) != hipSuccess)
            return fail(c, GF_E_NOMEM, "feature buffers");
        N.feat_cap = total;
    }
    if (!N.lv) HIPCHK(c, hipMalloc((void **)&N.lv, sizeof(gfnet::FeatLevel) * 16));
    const int m = c->m;
    int64_t row = 0;
    for (size_t si = 0; si < c->sc.size(); ++si) {
        const Scen &S = c->sc[si];
        if (S.leaves.empty()) continue;
        int Lf = 0;
        for (const Leaf &L : S.leaves) Lf = std::max(Lf, L.level);
        std::vector<gfnet::FeatLevel> lv((size_t)Lf + 1);
        int64_t moff = 0, ioff = 0;
        for (int l = 0; l <= Lf; ++l) {
            lv[l].map_off = moff;
            lv[l].map_w = S.d.mi << l;
            moff += (int64_t)(S.d.mi << l) * (S.d.mj << l);
            lv[l].img_off = ioff;
            lv[l].nx = 8 * (S.d.mi << l);
            lv[l].ny = 8 * (S.d.mj << l);
            ioff += 4 * (int64_t)lv[l].nx * lv[l].ny;
        }
        if (ioff > ((int64_t)1 << 28)) return fail(c, GF_E_UNSUPPORTED, "feature images too large for level %d", Lf);
        std::vector<int32_t> map((size_t)moff, -1);
        std::vector<int32_t> lij(S.leaves.size() * 3);
        for (size_t k = 0; k < S.leaves.size(); ++k) {
            const Leaf &L = S.leaves[k];
            map[(size_t)(lv[L.level].map_off + L.PJ * lv[L.level].map_w + L.PI)] = L.slot;
            lij[3 * k] = L.level;
            lij[3 * k + 1] = (int32_t)L.PI;
            lij[3 * k + 2] = (int32_t)L.PJ;
        }
        int64_t mc = (int64_t)N.map_cap, ic = (int64_t)N.img_cap;
        if (grow(&N.map, mc, moff) != hipSuccess || grow(&N.img, ic, ioff) != hipSuccess)
            return fail(c, GF_E_NOMEM, "feature images");
        N.map_cap = (size_t)mc;
        N.img_cap = (size_t)ic;
        if (grow(&N.lij, N.lij_cap, (int64_t)lij.size()) != hipSuccess) return fail(c, GF_E_NOMEM, "leaf table");
        HIPCHK(c, hipMemcpyAsync(N.map, map.data(), sizeof(int32_t) * map.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(N.lv, lv.data(), sizeof(gfnet::FeatLevel) * lv.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(N.lij, lij.data(), sizeof(int32_t) * lij.size(), hipMemcpyHostToDevice, c->stream));
        const int cur = c->hs[si].cur;
        hipError_t e;
        if (c->prec == GF_FP32)
            e = gfnet_launch_image_f32((const float *)c->q[cur], (const float *)c->b, c->cap, m, N.map, N.lv, lv[Lf], Lf,
                                       N.img, c->stream);
        else
            e = gfnet_launch_image_f64((const double *)c->q[cur], (const double *)c->b, c->cap, m, N.map, N.lv, lv[Lf],
                                       Lf, N.img, c->stream);
        for (int l = Lf - 1; l >= 0 && e == hipSuccess; --l)
            e = gfnet_launch_pyramid(N.img + lv[l + 1].img_off, lv[l + 1].nx, lv[l + 1].ny, N.img + lv[l].img_off,
                                     lv[l].nx, lv[l].ny, c->stream);
        if (e == hipSuccess)
            e = gfnet_launch_tiles(N.img, N.lv, N.lij, (int)S.leaves.size(), N.featf + row * gfnet::FEAT,
                                   N.featb + row * gfnet::FEAT, c->stream);
        if (e != hipSuccess) return fail(c, GF_E_HIP, "feature launch: %s", hipGetErrorString(e));
        HIPCHK(c, hipStreamSynchronize(c->stream));   // the staging tables are reused by the next scenario
        row += (int64_t)S.leaves.size();
    }
    if (n_out) *n_out = total;
    return GF_OK;
}

}  // namespace

int gf_net_set_params(gf_ctx *c, const double *params, int64_t n)
{
    if (!c || !params || n != gfnet::N_PARAMS) return GF_E_INVALID;
    auto &N = c->net;
    if (!N.w) {
        size_t b = sizeof(float) * gfnet::N_PARAMS;
        if (hipMalloc((void **)&N.w, b) != hipSuccess || hipMalloc((void **)&N.m, b) != hipSuccess ||
            hipMalloc((void **)&N.v, b) != hipSuccess || hipMalloc((void **)&N.g, b) != hipSuccess ||
            hipMalloc((void **)&N.wb, sizeof(uint16_t) * gfnet::N_PARAMS) != hipSuccess ||
            hipMalloc((void **)&N.wtot, 64) != hipSuccess)
            return fail(c, GF_E_NOMEM, "network parameters");
    }
    std::vector<float> w((size_t)n);
    for (int64_t i = 0; i < n; ++i) w[(size_t)i] = (float)params[i];
    HIPCHK(c, hipMemcpyAsync(N.w, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(N.m, 0, sizeof(float) * w.size(), c->stream));
    HIPCHK(c, hipMemsetAsync(N.v, 0, sizeof(float) * w.size(), c->stream));
    hipError_t e = gfnet_launch_to_bf16(N.w, N.wb, gfnet::N_PARAMS, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "weight conversion: %s", hipGetErrorString(e));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    N.t = 0;
    return GF_OK;
}

int gf_net_get_params(gf_ctx *c, double *out, int64_t n)
{
    if (!c || !out || n != gfnet::N_PARAMS) return GF_E_INVALID;
    int rc = net_ready(c);
    if (rc) return rc;
    std::vector<float> w((size_t)n);
    HIPCHK(c, hipMemcpyAsync(w.data(), c->net.w, sizeof(float) * w.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n; ++i) out[i] = w[(size_t)i];
    return GF_OK;
}

int gf_net_features(gf_ctx *c, double *out, int64_t cap, int64_t *n_leaves)
{
    if (!c) return GF_E_INVALID;
    for (auto &s : c->sc)
        if (!scen_ready(s)) return fail(c, GF_E_STATE, "scenario without bathymetry or leaves");
    int64_t n = 0;
    int rc = net_features(c, &n);
    if (rc) return rc;
    if (n_leaves) *n_leaves = n;
    if (!out) return GF_OK;
    if (cap < n * gfnet::FEAT) return fail(c, GF_E_INVALID, "feature buffer too small");
    std::vector<float> f((size_t)(n * gfnet::FEAT));
    HIPCHK(c, hipMemcpyAsync(f.data(), c->net.featf, sizeof(float) * f.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < f.size(); ++i) out[i] = f[i];
    return GF_OK;
}

int gf_net_forward(gf_ctx *c, const double *x, int32_t n, double *logits)
{
    if (!c || !x || !logits || n <= 0) return GF_E_INVALID;
    int rc = net_ready(c);
    if (rc) return rc;
    rc = net_stage_batch(c, x, n);
    if (rc) return rc;
    auto &N = c->net;
    gfnet::NetArgs a{};
    a.x = N.x; a.n = n; a.w = N.w; a.wb = N.wb; a.logits = N.logits;
    hipError_t e = gfnet_launch_forward(a, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "network launch: %s", hipGetErrorString(e));
    std::vector<float> z((size_t)n * 3);
    HIPCHK(c, hipMemcpyAsync(z.data(), N.logits, sizeof(float) * z.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < z.size(); ++i) logits[i] = z[i];
    return GF_OK;
}

int gf_net_train_step(gf_ctx *c, const double *x, const int8_t *y, int32_t n, const double *class_w, double lr,
                      double *loss, double *grad)
{
    if (!c || !x || !y || !class_w || n <= 0 || !(lr >= 0.0)) return GF_E_INVALID;
    int rc = net_ready(c);
    if (rc) return rc;
    double wtot = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        if (y[i] < 0 || y[i] > 2) return fail(c, GF_E_INVALID, "class label out of range");
        wtot += class_w[y[i]];
    }
    if (!(wtot > 0.0)) return fail(c, GF_E_INVALID, "class weights sum to zero over the batch");
    rc = net_stage_batch(c, x, n);
    if (rc) return rc;
    auto &N = c->net;
    HIPCHK(c, hipMemcpyAsync(N.y, y, (size_t)n, hipMemcpyHostToDevice, c->stream));
    gfnet::NetArgs a{};
    a.x = N.x; a.n = n; a.w = N.w; a.wb = N.wb; a.logits = N.logits;
    a.y = N.y; a.cw[0] = (float)class_w[0]; a.cw[1] = (float)class_w[1]; a.cw[2] = (float)class_w[2];
    a.wtot = (float)wtot; a.loss_i = N.loss; a.part = N.part;
    hipError_t e = gfnet_launch_train(a, c->stream);
    if (e == hipSuccess) e = gfnet_launch_reduce(N.part, n, N.g, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "training launch: %s", hipGetErrorString(e));
    if (grad) {
        std::vector<float> g(gfnet::N_PARAMS);
        HIPCHK(c, hipMemcpyAsync(g.data(), N.g, sizeof(float) * g.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < g.size(); ++i) grad[i] = g[i];
    }
    N.t += 1;
    const double bc1 = 1.0 - std::pow(0.9, (double)N.t), bc2 = 1.0 - std::pow(0.999, (double)N.t);
    e = gfnet_launch_adam(N.w, N.m, N.v, N.wb, N.g, (float)lr, (float)bc1, (float)bc2, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "optimiser launch: %s", hipGetErrorString(e));
    if (loss) {
        std::vector<float> li((size_t)n);
        HIPCHK(c, hipMemcpyAsync(li.data(), N.loss, sizeof(float) * li.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double L = 0.0;
        for (float v : li) L += v;
        *loss = L;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GF_OK;
}

int gf_net_train_step_dev(gf_ctx *c, const uint16_t *x_bf16, const int8_t *y, int32_t n, const double *class_w,
                          double lr, double *loss)
{
    if (!c) return GF_E_INVALID;
    if (!x_bf16 || !y || !class_w || n <= 0 || !(lr >= 0.0))
        return fail(c, GF_E_INVALID, "null batch pointer, empty batch or negative learning rate");
    int rc = net_ready(c);
    if (rc) return rc;
    rc = net_stage_batch(c, nullptr, n);
    if (rc) return rc;
    auto &N = c->net;
    hipError_t e = gfnet_launch_weight_sum(y, n, (float)class_w[0], (float)class_w[1], (float)class_w[2], N.wtot,
                                           c->stream);
    gfnet::NetArgs a{};
    a.x = nullptr; a.xb = x_bf16; a.n = n; a.w = N.w; a.wb = N.wb; a.logits = N.logits;
    a.y = y; a.cw[0] = (float)class_w[0]; a.cw[1] = (float)class_w[1]; a.cw[2] = (float)class_w[2];
    a.wtot = 0.f; a.wtot_dev = N.wtot; a.loss_i = N.loss; a.part = N.part;
    if (e == hipSuccess) e = gfnet_launch_train(a, c->stream);
    if (e == hipSuccess) e = gfnet_launch_reduce(N.part, n, N.g, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "training launch: %s", hipGetErrorString(e));
    N.t += 1;
    const double bc1 = 1.0 - std::pow(0.9, (double)N.t), bc2 = 1.0 - std::pow(0.999, (double)N.t);
    e = gfnet_launch_adam(N.w, N.m, N.v, N.wb, N.g, (float)lr, (float)bc1, (float)bc2, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "optimiser launch: %s", hipGetErrorString(e));
    if (loss) {
        std::vector<float> li((size_t)n);
        HIPCHK(c, hipMemcpyAsync(li.data(), N.loss, sizeof(float) * li.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double L = 0.0;
        for (float v : li) L += v;
        *loss = L;
    }
    return GF_OK;
}

int gf_net_predict(gf_ctx *c, int8_t *flags_out, int64_t cap, int64_t *n_out)
{
    if (!c) return GF_E_INVALID;
    int rc = net_ready(c);
    if (rc) return rc;
    for (auto &s : c->sc)
        if (!scen_ready(s)) return fail(c, GF_E_STATE, "scenario without bathymetry or leaves");
    int64_t n = 0;
    rc = net_features(c, &n);
    if (rc) return rc;
    rc = net_stage_batch(c, nullptr, (int32_t)n);
    if (rc) return rc;
    auto &N = c->net;
    gfnet::NetArgs a{};
    a.x = nullptr; a.xb = N.featb; a.n = (int)n; a.w = N.w; a.wb = N.wb; a.logits = N.logits;
    hipError_t e = gfnet_launch_forward(a, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "network launch: %s", hipGetErrorString(e));
    std::vector<float> z((size_t)n * 3);
    HIPCHK(c, hipMemcpyAsync(z.data(), N.logits, sizeof(float) * z.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // largest logit -> flag, within the scenario's level limits
    std::vector<int8_t> flags((size_t)n);
    int64_t k = 0;
    for (auto &S : c->sc)
        for (const Leaf &L : S.leaves) {
            const float *zz = &z[(size_t)(3 * k)];
            int cls = 1;
            if (zz[0] > zz[cls]) cls = 0;
            if (zz[2] > zz[cls]) cls = 2;
            int8_t f = (int8_t)(cls - 1);
            if (f > 0 && L.level >= S.d.max_level) f = 0;
            if (f < 0 && L.level <= S.d.min_level) f = 0;
            flags[(size_t)k++] = f;
        }
    c->last_flags.assign(flags.begin(), flags.end());
    if (n_out) *n_out = n;
    if (flags_out) {
        if (cap < n) return fail(c, GF_E_INVALID, "flag buffer too small");
        std::memcpy(flags_out, flags.data(), (size_t)n);
    }
    return GF_OK;
}

int gf_net_collect(gf_ctx *c, int32_t window, int32_t check_every, double *features, int8_t *labels, int64_t cap,
                   int64_t *n_out)
{
    if (!c || window <= 0 || check_every <= 0 || window % check_every) return GF_E_INVALID;
    for (auto &s : c->sc)
        if (!scen_ready(s)) return fail(c, GF_E_STATE, "scenario without bathymetry or leaves");
    int64_t n = 0;
    int rc = net_features(c, &n);
    if (rc) return rc;
    if (n_out) *n_out = n;
    if ((features || labels) && cap < n) return fail(c, GF_E_INVALID, "collect buffers too small (cap counts leaves)");
    if (features) {
        std::vector<float> f((size_t)(n * gfnet::FEAT));
        HIPCHK(c, hipMemcpyAsync(f.data(), c->net.featf, sizeof(float) * f.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < f.size(); ++i) features[i] = f[i];
    }
    // plain-tagger checks over the window on this leaf set
    std::vector<int8_t> any_refine((size_t)n, 0), all_coarsen((size_t)n, 1), fl((size_t)n);
    for (int32_t k = check_every; k <= window; k += check_every) {
        rc = gf_step(c, check_every, nullptr, nullptr);
        if (rc) return rc;
        int64_t nn = 0;
        rc = gf_tag(c, GF_TAG_PLAIN, fl.data(), n, &nn);
        if (rc) return rc;
        if (nn != n) return fail(c, GF_E_STATE, "leaf set changed during a collection window");
        for (int64_t i = 0; i < n; ++i) {
            any_refine[(size_t)i] |= fl[(size_t)i] > 0;
            all_coarsen[(size_t)i] &= fl[(size_t)i] < 0;
        }
    }
    std::vector<int8_t> lab((size_t)n);
    for (int64_t i = 0; i < n; ++i) lab[(size_t)i] = any_refine[(size_t)i] ? 1 : (all_coarsen[(size_t)i] ? -1 : 0);
    if (labels)
        for (int64_t i = 0; i < n; ++i) labels[i] = (int8_t)(lab[(size_t)i] + 1);
    int64_t nl = 0;
    return gf_regrid(c, lab.data(), &nl);
}

int gf_run(gf_ctx *c, int32_t nsteps, int32_t mode, int32_t check_every, int32_t regrid_every, gf_run_stats *out)
{
    if (!c || nsteps < 0 || check_every <= 0 || (mode != GF_RUN_PLAIN && (regrid_every <= 0 || regrid_every % check_every)))
        return GF_E_INVALID;
    if (mode < GF_RUN_PLAIN || mode > GF_RUN_LEARNED) return GF_E_INVALID;
    if (mode == GF_RUN_LEARNED) {
        int rc = net_ready(c);
        if (rc) return rc;
    }
    gf_run_stats st{};
    const auto t0 = std::chrono::steady_clock::now();
    auto n_leaves = [&]() {
        int64_t n = 0;
        for (auto &s : c->sc) n += (int64_t)s.leaves.size();
        return n;
    };
    std::vector<int8_t> plain, learned;
    int rc = GF_OK;
    for (int32_t k = 0; k < nsteps && rc == GF_OK; k += check_every) {
        const bool regrid_step = mode == GF_RUN_PLAIN || k % regrid_every == 0;
        int64_t n = n_leaves(), nn = 0;
        plain.resize((size_t)n);
        rc = gf_tag(c, GF_TAG_PLAIN, plain.data(), n, &nn);
        if (rc) break;
        if (regrid_step) {
            if (mode == GF_RUN_LEARNED) {
                learned.resize((size_t)n);
                rc = gf_net_predict(c, learned.data(), n, &nn);
                if (rc) break;
                // the plain tagger stays the reference: its refine requests always
                // hold, and a coarsening needs its agreement
                for (int64_t i = 0; i < n; ++i) {
                    int8_t f = learned[(size_t)i];
                    if (plain[(size_t)i] > 0) f = 1;
                    else if (f < 0 && plain[(size_t)i] >= 0) f = 0;
                    learned[(size_t)i] = f;
                }
                rc = gf_regrid(c, learned.data(), &nn);
            } else {
                rc = gf_regrid(c, plain.data(), &nn);
            }
            st.regrids += 1;
        } else {
            int64_t miss = 0;
            for (int64_t i = 0; i < n; ++i) miss += plain[(size_t)i] > 0;
            st.checks += n;
            st.misses += miss;
            if (miss && mode == GF_RUN_LEARNED) {
                for (auto &f : plain) f = f > 0 ? 1 : 0;
                rc = gf_regrid(c, plain.data(), &nn);
                st.forced_regrids += 1;
            }
        }
        if (rc) break;
        const int32_t ns = std::min(check_every, nsteps - k);
        gf_step_stats ss{};
        rc = gf_step(c, ns, nullptr, &ss);
        st.steps += ns;
        st.leaf_steps += n_leaves() * ns;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (out) *out = st;
    return rc;
}

int gf_mass(gf_ctx *c, int32_t scen, double *mass, double *clamp_volume, double *boundary_volume)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    rc = ensure_work(c);
    if (rc) return rc;
    const int nw = (int)c->desc.size();
    hipError_t e;
    if (c->prec == GF_FP32)
        e = gf_launch_mass_f32(c->d_desc, nw, c->d_scen, (const float *)c->q[0], (const float *)c->q[1], c->cap, c->d_mass, c->m, c->stream);
    else
        e = gf_launch_mass_f64(c->d_desc, nw, c->d_scen, (const double *)c->q[0], (const double *)c->q[1], c->cap, c->d_mass, c->m, c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "mass launch: %s", hipGetErrorString(e));
    std::vector<double> part((size_t)nw), ca((size_t)c->cap), ba((size_t)c->cap);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->d_mass, sizeof(double) * (size_t)nw, hipMemcpyDeviceToHost, c->stream));
    const int cur = c->hs[(size_t)scen].cur;
    HIPCHK(c, hipMemcpyAsync(ca.data(), c->cacc[cur], sizeof(double) * ca.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ba.data(), c->bacc[cur], sizeof(double) * ba.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double S = 0.0, C = 0.0, cl = c->sc[(size_t)scen].clamp_base, bd = c->sc[(size_t)scen].bnd_base;
    for (int k = 0; k < nw; ++k) {
        if (c->desc[(size_t)k].scen != scen) continue;
        const double v = part[(size_t)k], t = S + v;
        if (std::fabs(S) >= std::fabs(v)) C += (S - t) + v; else C += (v - t) + S;
        S = t;
        cl += ca[(size_t)c->desc[(size_t)k].slot];
        bd += ba[(size_t)c->desc[(size_t)k].slot];
    }
    if (mass) *mass = S + C;
    if (clamp_volume) *clamp_volume = cl;
    if (boundary_volume) *boundary_volume = bd;
    return GF_OK;
}

int gf_set_initial(gf_ctx *c, int32_t scen, gf_ic_fn ic, void *user, int32_t max_passes)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    if (!ic || max_passes < 0) return fail(c, GF_E_INVALID, "null initial-condition callback or negative pass count");
    Scen &S = c->sc[(size_t)scen];
    if (!scen_ready(S)) return fail(c, GF_E_STATE, "scenario without bathymetry or leaves");
    const int m = c->m;
    const size_t MM = (size_t)m * m;
    for (int pass = 0;; ++pass) {
        const size_t n = S.leaves.size();
        std::vector<double> st(n * 4 * MM), in(n * 3 * MM);
        rc = gf_get_state(c, scen, st.data());
        if (rc) return rc;
        for (size_t k = 0; k < n; ++k) {
            const Leaf &L = S.leaves[k];
            const double dx = (S.d.x1 - S.d.x0) / (double)(((int64_t)S.d.mi * m) << L.level);
            const double dy = (S.d.y1 - S.d.y0) / (double)(((int64_t)S.d.mj * m) << L.level);
            const double x0 = S.d.x0 + (double)(L.PI * m) * dx, y0 = S.d.y0 + (double)(L.PJ * m) * dy;
            ic(user, scen, L.level, x0, y0, dx, dy, m, m, &st[(k * 4 + 3) * MM], &in[(k * 3) * MM],
               &in[(k * 3 + 1) * MM], &in[(k * 3 + 2) * MM]);
        }
        rc = gf_set_state(c, scen, in.data());
        if (rc) return rc;
        if (pass >= max_passes) break;
        // the plain criteria on this scenario's leaves only
        int64_t nall = 0, off = 0;
        for (int32_t k = 0; k < scen; ++k) off += (int64_t)c->sc[(size_t)k].leaves.size();
        for (auto &s2 : c->sc) nall += (int64_t)s2.leaves.size();
        std::vector<int8_t> fl((size_t)nall);
        int64_t nn = 0;
        rc = gf_tag(c, GF_TAG_PLAIN, fl.data(), nall, &nn);
        if (rc) return rc;
        bool any = false;
        for (int64_t k = 0; k < nall; ++k) {
            if (k < off || k >= off + (int64_t)n) fl[(size_t)k] = 0;
            any = any || fl[(size_t)k] != 0;
        }
        if (!any) break;
        std::vector<uint64_t> before;
        for (const Leaf &L : S.leaves) before.push_back(key_of(L.level, L.PI, L.PJ));
        rc = gf_regrid(c, fl.data(), &nn);
        if (rc) return rc;
        std::vector<uint64_t> after;
        for (const Leaf &L : S.leaves) after.push_back(key_of(L.level, L.PI, L.PJ));
        if (after == before) break;
    }
    // the run starts here: clock, step count and budgets
    rc = fold_accumulators(c);
    if (rc) return rc;
    S.clamp_base = 0.0;
    S.bnd_base = 0.0;
    ScenDev &h = c->hs[(size_t)scen];
    h.t = 0.0; h.dt = 0.0; h.steps = 0; h.rejected = 0; h.status = 0; h.nu_max = 0.0;
    return push_scen(c);
}

int gf_mass_static(gf_ctx *c, int32_t scen, double *mass, double *clamp_volume, double *boundary_volume)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    if (c->static_err != hipSuccess || !c->static_scratch)
        return fail(c, GF_E_HIP, "static scratch unavailable: %s", hipGetErrorString(c->static_err));
    // the tables must be current: rebuilding them may allocate
    if (c->topo_dirty) return fail(c, GF_E_STATE, "mesh tables out of date (call gf_mass or gf_step once first)");
    const int nw = (int)c->desc.size();
    if (nw > gf::kStaticMassPatches)
        return fail(c, GF_E_INVALID, "%d patches exceed the static scratch of %d patches", nw, gf::kStaticMassPatches);
    double *part = c->static_scratch, *res = c->static_scratch + gf::kStaticMassPatches;
    hipError_t e = hipSuccess;
    if (nw > 0) {
        if (c->prec == GF_FP32)
            e = gf_launch_mass_f32(c->d_desc, nw, c->d_scen, (const float *)c->q[0], (const float *)c->q[1], c->cap, part,
                                   c->m, c->stream);
        else
            e = gf_launch_mass_f64(c->d_desc, nw, c->d_scen, (const double *)c->q[0], (const double *)c->q[1], c->cap,
                                   part, c->m, c->stream);
    }
    if (e != hipSuccess) return fail(c, GF_E_HIP, "mass launch: %s", hipGetErrorString(e));
    const int cur = c->hs[(size_t)scen].cur;
    const Scen &S = c->sc[(size_t)scen];
    e = gf_launch_mass_ordered(part, c->d_desc, nw, scen, c->cacc[cur], c->bacc[cur], S.clamp_base, S.bnd_base, res,
                               c->stream);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "mass sum launch: %s", hipGetErrorString(e));
    double out[3];
    HIPCHK(c, hipMemcpyAsync(out, res, sizeof out, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (mass) *mass = out[0];
    if (clamp_volume) *clamp_volume = out[1];
    if (boundary_volume) *boundary_volume = out[2];
    return GF_OK;
}

int gf_time(gf_ctx *c, int32_t scen, double *t, double *dt_next, int64_t *steps, int64_t *rejected)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    const ScenDev &h = c->hs[(size_t)scen];
    if (t) *t = h.t;
    if (dt_next) *dt_next = h.dt;
    if (steps) *steps = h.steps;
    if (rejected) *rejected = h.rejected;
    return GF_OK;
}

int gf_set_time(gf_ctx *c, int32_t scen, double t, double dt_next)
{
    int rc = check_scen(c, scen);
    if (rc) return rc;
    c->hs[(size_t)scen].t = t;
    c->hs[(size_t)scen].dt = dt_next;
    return push_scen(c);
}

int gf_set_step_threads(gf_ctx *c, int32_t nt)
{
    if (!c) return GF_E_INVALID;
    const int ok = c->prec == GF_FP32 ? gf_step_threads_ok_f32(c->m, nt) : gf_step_threads_ok_f64(c->m, nt);
    if (!ok) return fail(c, GF_E_UNSUPPORTED, "no step kernel built for m = %d with %d threads", c->m, nt);
    c->step_threads = nt;
    return GF_OK;
}

int gf_set_schedule(gf_ctx *c, int32_t workgroups)
{
    if (!c || workgroups < -1) return GF_E_INVALID;
    c->sched_wg = workgroups;
    return GF_OK;
}

int gf_set_step_pad(gf_ctx *c, int32_t pad)
{
    if (!c) return GF_E_INVALID;
    if (pad < 0 || pad > 1) return fail(c, GF_E_UNSUPPORTED, "no step kernel built with %d words of row padding", pad);
    c->step_pad = pad;
    return GF_OK;
}

int gf_autotune_trials(gf_ctx *c, int32_t *shapes, double *us, int64_t cap, int64_t *n)
{
    if (!c) return GF_E_INVALID;
    if (n) *n = (int64_t)c->tune_trials.size();
    if (!shapes && !us) return GF_OK;
    if (cap < (int64_t)c->tune_trials.size()) return fail(c, GF_E_INVALID, "trial buffer too small");
    for (size_t k = 0; k < c->tune_trials.size(); ++k) {
        const auto &t = c->tune_trials[k];
        if (shapes) { shapes[3 * k] = t.nt; shapes[3 * k + 1] = t.sched; shapes[3 * k + 2] = t.pad; }
        if (us) us[k] = t.us;
    }
    return GF_OK;
}

int gf_get_step_threads(gf_ctx *c, int32_t *nt)
{
    if (!c || !nt) return GF_E_INVALID;
    *nt = c->step_threads;
    return GF_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: time the step kernel's launch shapes on the context's own state
// and keep the fastest.  The state, clocks and accumulators are restored after
// every trial, so tuning does not change the simulation.
// ---------------------------------------------------------------------------
namespace {

// cache file: one line per key, "key threads sched us_per_step"
// cache lines: key threads schedule padding us_per_step
bool cache_lookup(const char *path, const std::string &key, int *nt, int *sched, int *pad)
{
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512], k[200];
    int a = 0, b = 0, d = 0;
    double us = 0.0;
    bool found = false;
    while (fgets(line, sizeof line, f))
        if (sscanf(line, "%199s %d %d %d %lf", k, &a, &b, &d, &us) == 5 && key == k) {
            *nt = a; *sched = b; *pad = d; found = true;
        }
    fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, int nt, int sched, int pad, double us)
{
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %.3f\n", key.c_str(), nt, sched, pad, us);
    fclose(f);
}

}  // namespace

int gf_set_gauges(gf_ctx *c, int32_t n, const int32_t *scen, const double *xy, int64_t cap)
{
    if (!c || n < 0 || n > kMaxGauges || (n > 0 && (!scen || !xy || cap < 1))) return GF_E_INVALID;
    std::vector<gf_ctx::GaugePoint> pts((size_t)n);
    for (int k = 0; k < n; ++k) {
        if (scen[k] < 0 || scen[k] >= (int)c->sc.size()) return fail(c, GF_E_INVALID, "gauge %d: no scenario %d", k, scen[k]);
        const gf_scenario_desc &d = c->sc[(size_t)scen[k]].d;
        const double x = xy[2 * k], y = xy[2 * k + 1];
        if (!(x >= d.x0 && x <= d.x1 && y >= d.y0 && y <= d.y1))
            return fail(c, GF_E_INVALID, "gauge %d: point outside its domain", k);
        pts[(size_t)k] = {scen[k], x, y};
    }
    if (c->d_gauges) { (void)hipFree(c->d_gauges); c->d_gauges = nullptr; }
    if (c->d_grec) { (void)hipFree(c->d_grec); c->d_grec = nullptr; }
    if (c->d_gcount) { (void)hipFree(c->d_gcount); c->d_gcount = nullptr; }
    c->gauges.clear();
    c->grec_cap = 0;
    if (n == 0) return GF_OK;
    HIPCHK(c, hipMalloc((void **)&c->d_gauges, sizeof(GaugeDev) * (size_t)n));
    HIPCHK(c, hipMalloc((void **)&c->d_grec, sizeof(double) * 5 * (size_t)n * (size_t)cap));
    HIPCHK(c, hipMalloc((void **)&c->d_gcount, sizeof(int64_t) * (size_t)n));
    HIPCHK(c, hipMemsetAsync(c->d_gcount, 0, sizeof(int64_t) * (size_t)n, c->stream));
    c->gauges = pts;
    c->grec_cap = cap;
    bool ready = true;
    for (auto &s : c->sc) ready = ready && scen_ready(s);
    if (!ready) return GF_OK;   // mapped when the mesh is built
    int rc = ensure_work(c);
    if (rc) return rc;
    return map_gauges(c);
}

int gf_get_gauges(gf_ctx *c, int32_t g, double *out, int64_t cap_out, int64_t *n)
{
    if (!c || g < 0 || g >= (int)c->gauges.size() || cap_out < 0 || (cap_out > 0 && !out)) return GF_E_INVALID;
    int64_t cnt = 0;
    HIPCHK(c, hipMemcpyAsync(&cnt, c->d_gcount + g, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (n) *n = cnt;
    const int64_t k = std::min(std::min(cnt, c->grec_cap), cap_out);
    if (k > 0) {
        HIPCHK(c, hipMemcpyAsync(out, c->d_grec + (size_t)g * (size_t)c->grec_cap * 5, sizeof(double) * 5 * (size_t)k,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return GF_OK;
}

int gf_autotune(gf_ctx *c, int32_t steps, const char *cache_path, int32_t *threads_out, int32_t *sched_out,
                int32_t *pad_out, double *us_per_step_out)
{
    if (!c || steps <= 0) return GF_E_INVALID;
    for (auto &s : c->sc)
        if (!scen_ready(s)) return fail(c, GF_E_STATE, "scenario without bathymetry or leaves");
    int rc = ensure_work(c);
    if (rc) return rc;
    const TuneKey key = tune_key(c);
    if (!cache_path && !c->tune_cache.empty()) cache_path = c->tune_cache.c_str();
    int best_nt = c->step_threads, best_sched = c->sched_wg, best_pad = c->step_pad;
    double best_us = -1.0;
    if (cache_lookup(cache_path, key.text, &best_nt, &best_sched, &best_pad)) {
        if (best_pad < 0 || best_pad > 1 || best_sched < -1) return fail(c, GF_E_INVALID, "bad autotune cache entry");
        rc = gf_set_step_threads(c, best_nt);
        if (rc) return rc;
        c->sched_wg = best_sched;
        c->step_pad = best_pad;
        if (threads_out) *threads_out = best_nt;
        if (sched_out) *sched_out = best_sched;
        if (pad_out) *pad_out = best_pad;
        if (us_per_step_out) *us_per_step_out = -1.0;
        return GF_OK;
    }
    // snapshot everything a step changes
    rc = pull_scen(c);
    if (rc) return rc;
    const std::vector<ScenDev> hs0 = c->hs;
    const size_t qbytes = 3 * (size_t)c->m * c->m * (size_t)c->cap * c->es;
    const size_t abytes = sizeof(double) * (size_t)c->cap;
    std::vector<std::pair<void *, size_t>> parts = {{c->q[0], qbytes}, {c->q[1], qbytes},
                                                    {c->cacc[0], abytes}, {c->cacc[1], abytes},
                                                    {c->bacc[0], abytes}, {c->bacc[1], abytes},
                                                    {c->dry[0], (size_t)c->cap}, {c->dry[1], (size_t)c->cap}};
    size_t total = 0;
    for (auto &p : parts) total += (p.second + 255) & ~(size_t)255;
    char *snap = nullptr;
    HIPCHK(c, hipMalloc((void **)&snap, total));
    auto copy_all = [&](bool save) -> hipError_t {
        size_t off = 0;
        for (auto &p : parts) {
            hipError_t e = save ? hipMemcpyAsync(snap + off, p.first, p.second, hipMemcpyDeviceToDevice, c->stream)
                                : hipMemcpyAsync(p.first, snap + off, p.second, hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return e;
            off += (p.second + 255) & ~(size_t)255;
        }
        return hipSuccess;
    };
    const bool flags_dirty0 = c->flags_dirty;
    const int nt0 = c->step_threads, sched0 = c->sched_wg, pad0 = c->step_pad;
    c->tune_trials.clear();
    const bool prof0 = c->prof;
    c->gauges_on = false;
    hipError_t e = copy_all(true);
    // shapes: workgroup size (cells per thread m^2 / threads) x LDS row
    // padding x schedule (the resident grid, half of it, one workgroup per
    // patch)
    static const int cand32[] = {256, 512, 1024}, cand16[] = {64, 128, 256};
    const int *cand = c->m == 16 ? cand16 : cand32;
    for (int ci = 0; ci < 3 && e == hipSuccess && rc == GF_OK; ++ci)
        for (int pad = 0; pad < 2 && e == hipSuccess && rc == GF_OK; ++pad)
            for (int si = 0; si < 3 && e == hipSuccess && rc == GF_OK; ++si) {
                c->step_threads = cand[ci];
                c->step_pad = pad;
                int sched = si == 0 ? -1 : 0;
                if (si == 1) {
                    const int res = c->prec == GF_FP32 ? gf_step_resident_f32(c->m, cand[ci], pad)
                                                       : gf_step_resident_f64(c->m, cand[ci], pad);
                    sched = std::max(1, res / 2);
                }
                c->sched_wg = sched;
                // one untimed step (first use of the shape), then the timed ones
                c->prof = false;
                rc = gf_step(c, 1, nullptr, nullptr);
                if (rc == GF_OK) {
                    c->prof = true;
                    c->prof_launches = 0;
                    c->prof_ms = 0.0;
                    rc = gf_step(c, steps, nullptr, nullptr);
                }
                int64_t n = 0;
                double ms = 0.0;
                if (rc == GF_OK) rc = gf_profile_read(c, &n, &ms);
                if (rc == GF_OK && n > 0) c->tune_trials.push_back({cand[ci], sched, pad, 1e3 * ms / (double)n});
                // restore
                c->hs = hs0;
                if ((e = copy_all(false)) != hipSuccess) break;
                int r2 = push_scen(c);
                if (rc == GF_OK) rc = r2;
                c->flags_dirty = flags_dirty0;
            }
    // the choice: the first trial (fewer threads, no padding, resident grid
    // first) within 2% of the fastest, so that shapes timed alike give the
    // same choice from run to run
    if (!c->tune_trials.empty()) {
        double fastest = c->tune_trials[0].us;
        for (const auto &t : c->tune_trials) fastest = std::min(fastest, t.us);
        for (const auto &t : c->tune_trials)
            if (t.us <= 1.02 * fastest) { best_us = t.us; best_nt = t.nt; best_sched = t.sched; best_pad = t.pad; break; }
    }
    c->prof = prof0;
    c->prof_launches = 0;
    c->prof_ms = 0.0;
    c->gauges_on = true;
    // the trials may have rewritten face records of patches the snapshot
    // holds as stable: every patch goes back to full dry updates
    if (e == hipSuccess) e = hipMemsetAsync(c->d_dstab, 0, (size_t)c->cap, c->stream);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(snap);
    if (e != hipSuccess) return fail(c, GF_E_HIP, "autotune snapshot: %s", hipGetErrorString(e));
    if (rc != GF_OK) { c->step_threads = nt0; c->sched_wg = sched0; c->step_pad = pad0; return rc; }
    c->step_threads = best_nt;
    c->sched_wg = best_sched;
    c->step_pad = best_pad;
    cache_store(cache_path, key.text, best_nt, best_sched, best_pad, best_us);
    if (threads_out) *threads_out = best_nt;
    if (sched_out) *sched_out = best_sched;
    if (pad_out) *pad_out = best_pad;
    if (us_per_step_out) *us_per_step_out = best_us;
    return GF_OK;
}

int gf_profile_patches(gf_ctx *c, int64_t *full_updates, int64_t *stable_dry)
{
    if (!c) return GF_E_INVALID;
    // [0] patches through the step kernel; [8 (1 + k)], k < 64: stable dry
    // patches counted by the dry kernel's workgroups k mod 64
    std::vector<unsigned long long> v(8 * 65, 0);
    HIPCHK(c, hipMemcpyAsync(v.data(), c->d_stats, sizeof(unsigned long long) * v.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    unsigned long long st = 0;
    for (int k = 1; k <= 64; ++k) st += v[8 * (size_t)k];
    if (full_updates) *full_updates = (int64_t)v[0];
    if (stable_dry) *stable_dry = (int64_t)st;
    return GF_OK;
}

int gf_profile_enable(gf_ctx *c, int32_t on)
{
    if (!c || on < 0 || on > 7) return GF_E_INVALID;
    if (c->prof_open) {
        int rc = prof_mark_end(c);
        if (rc) return rc;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        rc = prof_collect(c);
        if (rc) return rc;
    }
    if ((on & 1) && !c->prof) {
        c->prof_launches = 0;
        c->prof_ms = 0.0;
    }
    if ((on & 2) && !c->prof_stats) HIPCHK(c, hipMemsetAsync(c->d_stats, 0, 8 * 8 * 65, c->stream));
    c->prof = (on & 1) != 0;
    c->prof_stats = (on & 2) != 0;
    if ((on & 4) && !c->prof_kernel) c->kev_n = 0;
    c->prof_kernel = (on & 4) != 0;
    return GF_OK;
}

int gf_profile_kernel(gf_ctx *c, int64_t *launches, double *ms_total)
{
    if (!c) return GF_E_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (int64_t i = 0; i < c->kev_n; ++i) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->kev[2 * (size_t)i], c->kev[2 * (size_t)i + 1]));
        sum += ms;
    }
    if (launches) *launches = c->kev_n;
    if (ms_total) *ms_total = sum;
    c->kev_n = 0;
    return GF_OK;
}

int gf_profile_read(gf_ctx *c, int64_t *launches, double *ms_total)
{
    if (!c) return GF_E_INVALID;
    int rc = prof_mark_end(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    rc = prof_collect(c);
    if (rc) return rc;
    if (launches) *launches = c->prof_launches;
    if (ms_total) *ms_total = c->prof_ms;
    c->prof_launches = 0;
    c->prof_ms = 0.0;
    return GF_OK;
}

}  // extern "C"
