// Host runtime behind include/bqs.h: argument checks, workspace layout,
// kernel selection and the drivers of the recursion levels.
//
// The Quicksort main loop of the paper (Algorithm 1 with an explicit stack,
// Section 2) becomes a breadth-first sequence of recursion levels: all
// segments of one level are partitioned by one launch, their children form
// the next level's list on the device.  Segments of at most small_cut keys
// leave the loop and are sorted in LDS; runs of keys equal to a pivot leave
// it as well (the pivot is excluded from the recursion, Section 2).
//
// Default (asynchronous) mode: a call enqueues the levels with grids sized
// from device-side counts -- each kernel reads its level's counts from the
// control block and surplus workgroups leave at once -- for as many levels
// as the input is expected to need, then one single-workgroup launch that
// finishes whatever recursion is left, then a copy of the control block's
// counters to pinned host memory and an event.  Nothing waits: the call
// returns once the work is enqueued, and the counters are read when the
// event has passed (statistics, latched errors, the depth the next call of
// the same shape enqueues).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "bqs.h"
#include "bqs_internal.h"

namespace bqs {

// ---------------------------------------------------------------- set-up --

// Clears the control block (workgroup of 64 threads).
__device__ void clear_ctl(Ctl* c) {
    const int t = threadIdx.x;
    for (int i = t; i < kLevelStats; i += 64) c->level_keys[i] = 0;
    for (int x = t; x < kMaxXcd; x += 64) {
        c->xcd_arrive[x][0] = 0;
        c->xcd_n[x] = 0;
    }
    if (t == 0) {
        for (int s = 0; s < 2; ++s) {
            c->lc[s].segs = 0;
            c->lc[s].fills = 0;
            for (int k = 0; k < kSmallClasses; ++k) c->lc[s].smalls[k] = 0;
            c->lc[s].tile_next = 0;
            c->lc[s].tab = 0;
            c->lc[s].keys = 0;
        }
        c->error = 0;
        c->levels = 0;
        c->part_keys = c->small_keys = c->fill_keys = c->tiles = 0;
        for (int i = 0; i < 8; ++i) c->prof[i] = 0;
        for (int i = 0; i < 8; ++i) c->sprof[i] = 0;
        c->bar_arrive = 0;
        c->bar_gen = 0;
    }
}

// Single array: the whole array is level 0's only segment (or one small
// segment).
__global__ __launch_bounds__(64) void k_init_single(Args a) {
    Ctl* c = a.ctl;
    clear_ctl(c);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int64_t n = a.n;
    if (n > a.small_cut) {
        const int64_t T = a.tile_keys;
        const uint32_t nt = seg_tiles(0, n, T);
        SegDesc d{};
        d.lo = 0;
        d.hi = n;
        d.t0 = 0;
        d.nt = nt;
        a.segs[0][0] = d;
        c->lc[0].segs = (static_cast<unsigned long long>(nt) << 32) | 1ull;
        c->part_keys = static_cast<unsigned long long>(n);
        c->lc[0].keys = static_cast<unsigned long long>(n);
        c->level_keys[0] = static_cast<unsigned long long>(n);
        c->tiles = nt;
    } else if (n >= 2) {
        const int cls = small_class(n);
        a.smalls[0][static_cast<size_t>(cls) * a.cap_small] = SmallItem{0, n, 0u, 0u};
        c->lc[0].smalls[cls] = 1;
    }
}

__global__ __launch_bounds__(64) void k_zero_ctl(Args a) {
    clear_ctl(a.ctl);
    if (a.ticks && threadIdx.x == 0) a.ticks[a.k] = wall_clock64();  // segmented calls: the start
}

// One thread per segment: validate the offsets, then route the segment to
// the level-0 partition list or straight to the small sort.
__global__ __launch_bounds__(256) void k_init_segments(Args a) {
    __shared__ unsigned long long s_keys, s_tiles;
    if (threadIdx.x == 0) s_keys = s_tiles = 0;
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    Ctl* c = a.ctl;
    if (i < a.k) {
        const int64_t lo = a.offsets[i], hi = a.offsets[i + 1];
        const bool bad = lo < 0 || hi < lo || hi > a.n || (i == 0 && lo != 0) ||
                         (i == a.k - 1 && hi != a.n) || hi - lo >= (int64_t(1) << 31);
        const int64_t m = hi - lo;
        // completion clock: a segment of at most one key is final already;
        // the others' times are raised by the kernels that finish their pieces
        if (a.ticks) a.ticks[i] = bad || m > 1 ? 0ull : a.ticks[a.k];
        if (bad) {
            atomicOr(&c->error, ERR_OFFSETS);
        } else if (m > a.small_cut) {
            const int64_t T = a.tile_keys;
            const uint32_t nt = seg_tiles(lo, hi, T);
            const unsigned long long r =
                atomicAdd(&c->lc[0].segs, (static_cast<unsigned long long>(nt) << 32) | 1ull);
            const uint32_t idx = static_cast<uint32_t>(r);
            const uint64_t t0 = r >> 32;
            if (idx >= a.cap_seg || t0 + nt > a.cap_tile) {
                atomicOr(&c->error, ERR_OVERFLOW);
            } else {
                SegDesc d{};
                d.lo = lo;
                d.hi = hi;
                d.t0 = static_cast<uint32_t>(t0);
                d.nt = nt;
                d.origin = static_cast<uint32_t>(i);
                a.segs[0][idx] = d;
                atomicAdd(&s_keys, static_cast<unsigned long long>(m));
                atomicAdd(&s_tiles, static_cast<unsigned long long>(nt));
            }
        } else if (m >= 2) {
            const int cls = small_class(m);
            const uint32_t idx = atomicAdd(&c->lc[0].smalls[cls], 1u);
            if (idx >= a.cap_small) atomicOr(&c->error, ERR_OVERFLOW);
            else a.smalls[0][static_cast<size_t>(cls) * a.cap_small + idx] = SmallItem{lo, hi, static_cast<uint32_t>(i), 0u};
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_keys) {
        atomicAdd(&c->part_keys, s_keys);
        atomicAdd(&c->lc[0].keys, s_keys);
        atomicAdd(&c->level_keys[0], s_keys);
        atomicAdd(&c->tiles, s_tiles);
    }
}

// Map kernel, level L: one thread per tile finds the tile's segment (the
// segment list is ordered by first tile) and writes the tile descriptor;
// it also clears the tile's look-back status word.
__global__ __launch_bounds__(256) void k_map(Args a) {
    if (a.ctl->error) return;  // an earlier step latched an error: the rest of the call does nothing
    map_tiles(a, a.level, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// Check mode: latches ERR_NAN if any floating-point key is a NaN (exponent
// all ones, fraction not zero).  `wide`: 8-byte keys.  Runs after the init
// kernel has cleared the error word and before any level, and only reads.
__global__ __launch_bounds__(256) void k_check_nan(const void* keys, int64_t n, int wide, Ctl* c) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    bool nan = false;
    if (wide) {
        const uint64_t* k = static_cast<const uint64_t*>(keys);
        for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
            nan |= (k[i] & 0x7fffffffffffffffull) > 0x7ff0000000000000ull;
    } else {
        const uint32_t* k = static_cast<const uint32_t*>(keys);
        for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
            nan |= (k[i] & 0x7fffffffu) > 0x7f800000u;
    }
    if (__ballot(nan) && (threadIdx.x & 63) == 0) atomicOr(&c->error, ERR_NAN);
}

// ------------------------------------------------------------- records --
// The paper's large element types (Section 4, experimental setup), sorted as
// (key, index) pairs and then gathered.  Vector: ten doubles ordered by the
// sum of the squares of the components, summed left to right with every
// product and sum rounded (no fused multiply-add), as the comparison
// computes it.  Record: 21 int32 ordered by the first component.

__global__ __launch_bounds__(256) void k_vector_keys(const double* in, int64_t n, double* keys, uint32_t* idx) {
#pragma clang fp contract(off)
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* v = in + i * 10;
    double s = v[0] * v[0];
#pragma unroll
    for (int k = 1; k < 10; ++k) s = s + v[k] * v[k];
    keys[i] = s;
    idx[i] = static_cast<uint32_t>(i);
}

__global__ __launch_bounds__(256) void k_record_keys(const int32_t* in, int64_t n, int32_t* keys, uint32_t* idx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = in[i * 21];
    idx[i] = static_cast<uint32_t>(i);
}

// out record i = in record idx[i], one 4-byte word per thread (W words per
// record): consecutive threads write consecutive words.
__global__ __launch_bounds__(256) void k_gather_words(const uint32_t* in, const uint32_t* idx, int64_t n, int W,
                                                      uint32_t* out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t x = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; x < n * W; x += stride) {
        const int64_t i = x / W;
        const int w = static_cast<int>(x - i * W);
        out[x] = in[static_cast<int64_t>(idx[i]) * W + w];
    }
}

void launch_map(const Args& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_map, dim3(grid), dim3(256), 0, s, a);
}

void launch_init_single(const Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_init_single, dim3(1), dim3(64), 0, s, a);
}

void launch_init_segments(const Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_ctl, dim3(1), dim3(64), 0, s, a);
    const int64_t blocks = (a.k + 255) / 256;
    if (blocks > 0) hipLaunchKernelGGL(k_init_segments, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a);
}

// -------------------------------------------------------------- layout ----

struct Layout {
    size_t ctl, yk, yv, side, segs[2], smalls[2], fills[2], tile_desc, status, total;
    size_t splitters[2], toff, bcur, bstart;
    size_t ipmask, iptile, iprank;
    uint64_t cap_tab;
    uint64_t cap_seg, cap_tile, cap_small, cap_fill;
};

static size_t align_up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Workspace layout: the control block, the double buffer (keys, payloads
// and the side buffer for payloads of pivot-equal keys) and the per-level
// work lists in two slots.  In-place levels have no double buffer: one
// class bit per key (per tile of kIpT keys) and per-tile counts instead.
static Layout make_layout(int64_t n, size_t kb, size_t vb, int64_t k, int64_t T, int64_t S, bool multiway,
                          bool inplace) {
    Layout L{};
    const uint64_t un = static_cast<uint64_t>(n);
    const uint64_t uk = static_cast<uint64_t>(k);
    const uint64_t per_level_segs = un / static_cast<uint64_t>(S + 1) + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.ctl = take(sizeof(Ctl));
    L.yk = take(inplace ? 0 : un * kb);
    L.yv = take(vb && !inplace ? un * vb : 0);
    L.side = take(vb && !inplace ? un * vb : 0);
    // a two-way level gives each segment two children and one equal run;
    // a multiway level up to 16 children and 15 equal runs
    const uint64_t fan = multiway ? 16 : 2;
    L.cap_seg = per_level_segs;
    L.cap_tile = un / static_cast<uint64_t>(T) + 2 * L.cap_seg + 2;
    L.cap_small = fan * L.cap_seg + uk + 2;
    L.cap_fill = (fan - 1) * L.cap_seg + 1;
    for (int s = 0; s < 2; ++s) L.segs[s] = take(L.cap_seg * sizeof(SegDesc));
    for (int s = 0; s < 2; ++s) L.smalls[s] = take(kSmallClasses * L.cap_small * sizeof(SmallItem));
    for (int s = 0; s < 2; ++s) L.fills[s] = take(L.cap_fill * sizeof(FillItem));
    L.tile_desc = take(L.cap_tile * sizeof(TileDesc));
    L.status = take(L.cap_tile * sizeof(unsigned long long));
    // multiway levels: 16 splitters, 32 bucket cursors and 32 bucket
    // starts per segment, 32 bucket offsets per tile
    const bool mw = multiway && !inplace;
    for (int s = 0; s < 2; ++s) L.splitters[s] = take(mw ? L.cap_seg * 16 * sizeof(uint64_t) : 0);
    L.toff = take(mw ? L.cap_tile * 32 * sizeof(uint32_t) : 0);
    L.bcur = take(mw ? L.cap_seg * 32 * sizeof(uint32_t) : 0);
    L.bstart = take(mw ? L.cap_seg * 32 * sizeof(uint32_t) : 0);
    L.ipmask = take(inplace ? L.cap_tile * kIpWords * sizeof(uint64_t) : 0);
    L.iptile = take(inplace ? L.cap_tile * sizeof(IpTile) : 0);
    L.cap_tab = inplace ? un / kIpRankStep + 2 * L.cap_seg + 2 : 0;
    L.iprank = take(L.cap_tab * sizeof(uint32_t));
    L.total = off;
    return L;
}

static size_t key_bytes(int dtype) {
    switch (dtype) {
        case BQS_I32: case BQS_U32: case BQS_F32: return 4;
        case BQS_I64: case BQS_U64: case BQS_F64: return 8;
        default: return 0;
    }
}

}  // namespace bqs

// ----------------------------------------------------------------- ctx ----

struct bqs_ctx {
    hipStream_t stream = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int64_t small_cut = 0;
    int64_t sample_max = 0;
    int64_t pivot_mode = 0;
    int64_t pivot_skew = 0;
    int64_t timing = 0;
    int64_t ept = 0;
    int64_t grid = 0;
    int64_t profile = 0;
    int64_t mode = BQS_MODE_ASYNC;
    int64_t graph = 0;
    int64_t lookback = 0;   // 1: keys-only tiles also claim by decoupled look-back
    int64_t multiway = 0;   // 1: keys-only levels split around up to 15 splitters
    int64_t inplace = 0;    // 1: in-place levels (no double buffer)
    unsigned long long* ticks = nullptr;  // segmented calls' completion clock (caller's device array)
    int64_t ticks_count = 0;
    int64_t check_nan = 0;  // 1: floating-point keys are checked for NaN first
    int64_t enqueue_levels = 0;  // > 0: levels enqueued before the tail launch
    int64_t depth_limit = 0;     // > 0: replaces 2 floor(log2 n) + 3
    int64_t list_cap = 0;        // > 0: caps the per-level list capacities (stress test)
    int64_t shuffle = 0;         // 1: out-of-order tile claims and delayed look-back publication
    // graph mode: the captured launch sequence and the call shape it belongs to
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph_obj = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> gkey;
    int glevels = 0;
    int64_t persist_grid = 0;  // resident workgroups of the persistent kernel (cached per table)
    const void* persist_ops = nullptr;
    // results of the most recent call that has completed
    bqs_stats stats{};
    std::vector<int64_t> level_keys;
    std::vector<double> level_ms;
    bqs_status latched = BQS_OK;  // first device-detected error since the last bqs_ctx_sync_status
    // host-driven mode: control block read back between levels
    bqs::Ctl* pinned = nullptr;
    // calls in flight: the copy of their control block, the event that
    // follows it, and what the host knows of the call
    struct Done {
        bqs::Ctl* slot;
        hipEvent_t ev;
        uint64_t call;
        std::vector<uint64_t> shape;
        bqs_stats host;  // fields the host sets (tile size, cutoff, launches)
    };
    std::deque<Done> inflight;
    std::vector<bqs::Ctl*> free_slots;
    uint64_t calls = 0;
    // levels that calls of a given shape partitioned (from completed calls)
    std::map<std::vector<uint64_t>, int> seen_levels;
    // timing: event pairs recorded around launches, resolved when their call
    // has completed
    std::vector<hipEvent_t> ev_pool;
    struct Pending {
        hipEvent_t a, b;
        int kind;  // 0 plan, 1 small, 2 partition
        int level;
        uint64_t call;
    };
    std::vector<Pending> pending;
};

using namespace bqs;

namespace {

const Ops* select_ops(const bqs_ctx* ctx, int dtype, int val_bytes) {
    if (val_bytes == 0) return ops_keys(dtype, ctx ? static_cast<int>(ctx->ept) : 0);
    if (val_bytes == 4) return ops_pairs32(dtype);
    if (val_bytes == 8) return ops_pairs64(dtype);
    return nullptr;
}

// Keys per partition tile of a call: the multiway levels have their own.
int64_t eff_tile_keys(const bqs_ctx* ctx, const Ops* o) {
    if (ctx && ctx->inplace) return kIpT;
    return ctx && ctx->multiway && o->mscan ? o->multi_tile_keys : o->tile_keys;
}

// Smallest tile a call may use (it sizes the tile lists): the two-way
// keys-only levels of enqueued calls take half-size tiles on levels of many
// segments.
int64_t layout_tile_keys(const bqs_ctx* ctx, const Ops* o) {
    const int64_t t = eff_tile_keys(ctx, o);
    const bool two_way = !(ctx && (ctx->inplace || (ctx->multiway && o->mscan)));
    return two_way && o->half_tile_keys > 0 ? std::min<int64_t>(t, o->half_tile_keys) : t;
}

int64_t eff_small_cut(const bqs_ctx* ctx, const Ops* o) {
    int64_t s = ctx && ctx->small_cut > 0 ? ctx->small_cut : o->small_default;
    if (s > o->small_max) s = o->small_max;
    if (ctx && ctx->mode == BQS_MODE_PERSISTENT && s > o->persist_small_max) s = o->persist_small_max;
    if (s < 2) s = 2;
    return s;
}

int64_t floor_log2(int64_t n) {
    int64_t k = 0;
    while (n > 1) {
        n >>= 1;
        ++k;
    }
    return k;
}

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
    if (!a || !b || !an || !bn) return false;
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bn && y < x + an;
}

bqs_status hip_ok(hipError_t e) { return e == hipSuccess ? BQS_OK : BQS_EHIP; }

// Bytes of the control block the host reads: counters, status and per-level
// statistics; the barrier lines of the persistent mode stay on the device.
constexpr size_t kCtlHostBytes = offsetof(Ctl, bar_arrive);

hipEvent_t take_event(bqs_ctx* ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Event pairs around launches of call `call`.
struct Timer {
    bqs_ctx* ctx;
    bool on;           // partition passes are timed
    bool all;          // every other launch too
    uint64_t call;
    hipStream_t s;
    hipEvent_t a = nullptr;
    void start_aux() {
        if (all) start();
    }
    void stop_aux(int kind, int level) {
        if (all) stop(kind, level);
    }
    void start() {
        if (!on) return;
        a = take_event(ctx);
        if (a && hipEventRecord(a, s) != hipSuccess) {
            ctx->ev_pool.push_back(a);
            a = nullptr;
        }
    }
    void stop(int kind, int level) {
        if (!on || !a) return;
        hipEvent_t b = take_event(ctx);
        if (!b || hipEventRecord(b, s) != hipSuccess) {
            ctx->ev_pool.push_back(a);
            if (b) ctx->ev_pool.push_back(b);
            a = nullptr;
            return;
        }
        ctx->pending.push_back({a, b, kind, level, call});
        a = nullptr;
    }
};

// Adds the timings of call `call` (all of its events have completed) to
// `st` and the per-level times.
void resolve_events(bqs_ctx* ctx, uint64_t call, bqs_stats& st, std::vector<double>& level_ms) {
    std::vector<bqs_ctx::Pending> keep;
    for (auto& p : ctx->pending) {
        if (p.call != call) {
            keep.push_back(p);
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) ms = 0.f;
        if (p.kind == 0) st.plan_ms += ms;
        else if (p.kind == 1) st.small_ms += ms;
        else {
            st.partition_ms += ms;
            if (p.level >= 0) {
                if (level_ms.size() <= static_cast<size_t>(p.level)) level_ms.resize(p.level + 1, 0.0);
                level_ms[p.level] += ms;
            }
        }
        ctx->ev_pool.push_back(p.a);
        ctx->ev_pool.push_back(p.b);
    }
    ctx->pending.swap(keep);
}

void fill_stats(bqs_stats& stats, const Ctl& c) {
    stats.levels = static_cast<int64_t>(c.levels);
    stats.partitioned_keys = static_cast<int64_t>(c.part_keys);
    stats.small_sorted_keys = static_cast<int64_t>(c.small_keys);
    stats.filled_keys = static_cast<int64_t>(c.fill_keys);
    stats.tiles = static_cast<int64_t>(c.tiles);
    stats.prof_tiles = static_cast<int64_t>(c.prof[0]);
    stats.prof_lookback_rounds = static_cast<int64_t>(c.prof[1]);
    stats.prof_lookback_polls = static_cast<int64_t>(c.prof[2]);
    stats.prof_lookback_cycles = static_cast<double>(c.prof[3]);
    stats.prof_tile_cycles = static_cast<double>(c.prof[4]);
    stats.prof_load_cycles = static_cast<double>(c.prof[5]);
    stats.prof_small_segments = static_cast<int64_t>(c.sprof[0]);
    for (int i = 0; i < 5; ++i) stats.prof_small_cycles[i] = static_cast<double>(c.sprof[1 + i]);
}

void latch(bqs_ctx* ctx, bqs_status st) {
    if (st != BQS_OK && ctx->latched == BQS_OK) ctx->latched = st;
}

// Folds in the calls that have completed, oldest first (all of them, waiting
// as needed, with `wait`): latched error, statistics, per-level figures and
// the depth each call shape needed.
void harvest(bqs_ctx* ctx, bool wait) {
    while (!ctx->inflight.empty()) {
        bqs_ctx::Done& d = ctx->inflight.front();
        if (wait) {
            if (hipEventSynchronize(d.ev) != hipSuccess) latch(ctx, BQS_EHIP);
        } else {
            const hipError_t q = hipEventQuery(d.ev);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) latch(ctx, BQS_EHIP);
        }
        const Ctl& c = *d.slot;
        latch(ctx, status_of_device_error(c.error));
        bqs_stats st = d.host;
        fill_stats(st, c);
        std::vector<double> lms;
        resolve_events(ctx, d.call, st, lms);
        const int nl = static_cast<int>(std::min<int64_t>(st.levels, kLevelStats));
        ctx->level_keys.assign(c.level_keys, c.level_keys + nl);
        lms.resize(nl, 0.0);
        ctx->level_ms = lms;
        ctx->stats = st;
        if (!c.error) ctx->seen_levels[d.shape] = static_cast<int>(c.levels);
        ctx->free_slots.push_back(d.slot);
        ctx->ev_pool.push_back(d.ev);
        ctx->inflight.pop_front();
    }
}

// Records the end of an enqueued call: its control block is copied to a
// pinned slot, then an event.
bqs_status record_completion(bqs_ctx* ctx, const Args& a, hipStream_t s, uint64_t call,
                             const std::vector<uint64_t>& shape, const bqs_stats& host) {
    harvest(ctx, false);
    if (ctx->inflight.size() >= 64) harvest(ctx, true);  // bounds the pinned slots a context holds
    Ctl* slot = nullptr;
    if (!ctx->free_slots.empty()) {
        slot = ctx->free_slots.back();
        ctx->free_slots.pop_back();
    } else {
        void* p = nullptr;
        if (hipHostMalloc(&p, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return BQS_EHIP;
        slot = static_cast<Ctl*>(p);
    }
    hipEvent_t ev = take_event(ctx);
    if (!ev || hipMemcpyAsync(slot, a.ctl, kCtlHostBytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess) {
        ctx->free_slots.push_back(slot);
        if (ev) ctx->ev_pool.push_back(ev);
        return BQS_EHIP;
    }
    ctx->inflight.push_back({slot, ev, call, shape, host});
    return BQS_OK;
}

int clamp_grid(uint64_t want, int64_t cap) {
    if (want < 1) want = 1;
    if (want > static_cast<uint64_t>(cap)) want = static_cast<uint64_t>(cap);
    return static_cast<int>(want);
}

// The shape of a call: what its launch sequence depends on.
std::vector<uint64_t> call_shape(const Ops* o, const Args& a, bool segmented) {
    auto u = [](const void* p) { return static_cast<uint64_t>(reinterpret_cast<uintptr_t>(p)); };
    return {u(o), static_cast<uint64_t>(a.n), static_cast<uint64_t>(a.k), static_cast<uint64_t>(a.small_cut),
            static_cast<uint64_t>(a.sample_max), static_cast<uint64_t>(a.pivot_mode),
            static_cast<uint64_t>(a.pivot_skew), static_cast<uint64_t>(a.tile_keys), static_cast<uint64_t>(a.prof),
            static_cast<uint64_t>(a.claim), static_cast<uint64_t>(a.ways), static_cast<uint64_t>(a.depth_limit),
            static_cast<uint64_t>(a.shuffle), static_cast<uint64_t>(a.cap_seg), static_cast<uint64_t>(a.cap_small),
            static_cast<uint64_t>(a.inplace), segmented ? 1ull : 0ull};
}

// Graph key: the shape plus the buffers the launches were captured with.
std::vector<uint64_t> graph_key(const Ops* o, const Args& a, bool segmented, bool check) {
    auto u = [](const void* p) { return static_cast<uint64_t>(reinterpret_cast<uintptr_t>(p)); };
    std::vector<uint64_t> k = call_shape(o, a, segmented);
    for (uint64_t v : {u(a.ctl), u(a.x_keys), u(a.x_vals), u(a.y_keys), u(a.offsets), u(a.ticks),
                       uint64_t(check ? 1 : 0)})
        k.push_back(v);
    return k;
}

int level_cap(const Args& a) { return 4 * a.depth_limit + 64; }

// Levels a call enqueues before its tail launch: the levels that the last
// completed call of the same shape partitioned, plus its final level and
// one spare; for a new shape, an estimate from the largest possible segment
// (about log2(n / small_cut) halvings with sampled pivots, or a quarter as
// many sixteen-way splits) with some spare levels.
int estimate_levels(const Args& a) {
    int L = 1;
    if (a.n > a.small_cut) {
        const double r = std::log2(static_cast<double>(a.n) / static_cast<double>(a.small_cut));
        L = a.ways ? static_cast<int>(std::ceil(r / 4.0)) + 3 : static_cast<int>(std::ceil(r)) + 5;
    }
    return std::max(1, std::min(L, level_cap(a)));
}

int levels_to_enqueue(const bqs_ctx* ctx, const Args& a, const std::vector<uint64_t>& shape) {
    if (ctx->enqueue_levels > 0) return static_cast<int>(std::min<int64_t>(ctx->enqueue_levels, 1 << 20));
    const auto it = ctx->seen_levels.find(shape);
    if (it == ctx->seen_levels.end()) return estimate_levels(a);
    return std::max(1, std::min(it->second + 2, level_cap(a)));
}

// Most segments level L can hold: k at level 0, times the fan-out per level
// (two children, or up to sixteen for a multiway level), at most cap_seg.
uint64_t seg_bound(const Args& a, int L) {
    const uint64_t fan = a.ways ? 16 : 2;
    uint64_t segs = static_cast<uint64_t>(std::max<int64_t>(a.k, 1));
    for (int i = 0; i < L && segs < a.cap_seg; ++i) segs *= fan;
    return std::min<uint64_t>(segs, a.cap_seg);
}

// Two-way keys-only levels whose segment bound reaches this take half-size
// tiles (on 2^28 int32 keys: from level 8 on, 378-391 us a full level
// against 403-410 us; with fewer segments the claims of the many small tiles
// crowd onto few cursors, 818 us at level 0).
constexpr uint64_t kHalfTileSegs = 256;
// Levels of fewer segments take double-size tiles on 512 threads when the
// array fills at least kDoubleTileMin of them (the first levels of 2^28
// int32 keys: about 425 us a level against 450 us, half the claims on their
// one to sixteen cursors).
constexpr uint64_t kDoubleTileSegs = 32;
constexpr uint64_t kDoubleTileMin = 2048;

// Most tiles level L can hold: its segments are disjoint, and each has at
// most one partial tile, so n/T plus one per segment.
uint64_t tile_bound(const Args& a, int L) {
    const uint64_t T = static_cast<uint64_t>(a.tile_keys);
    return std::min<uint64_t>(static_cast<uint64_t>(a.n) / T + seg_bound(a, L) + 2, a.cap_tile);
}

// Enqueues init, the optional NaN check, `levels` recursion levels with
// grids that cover the most work each level can hold (the kernels read the
// actual counts on the device), and the tail launch.  `tm` may be null (no
// timing, e.g. under graph capture).
bqs_status enqueue_levels(const Ops* o, Args a, bool segmented, bool check, int dtype, int levels,
                          hipStream_t s, Timer* tm) {
    const bool alt = o->half_tile_keys > 0 && !a.ways && !a.inplace && a.claim != 0 && !a.shuffle;
    // (the last three enqueued levels carry little work, or none when the
    // learned depth holds: their launches stay small with the default tiles)
    auto tile_keys_of = [&](int L) {
        if (!alt || L + 3 >= levels) return o->tile_keys;
        const uint64_t sb = seg_bound(a, L);
        if (sb >= kHalfTileSegs) return o->half_tile_keys;
        if (sb < kDoubleTileSegs && static_cast<uint64_t>(a.n) / o->double_tile_keys >= kDoubleTileMin)
            return o->double_tile_keys;
        return o->tile_keys;
    };
    if (!a.ways && !a.inplace) a.tile_keys = tile_keys_of(0);
    if (segmented) launch_init_segments(a, s);
    else launch_init_single(a, s);
    if (check && (dtype == BQS_F32 || dtype == BQS_F64))
        hipLaunchKernelGGL(k_check_nan, dim3(clamp_grid((a.n + 255) / 256, 2048)), dim3(256), 0, s, a.x_keys, a.n,
                           dtype == BQS_F64 ? 1 : 0, a.ctl);
    const uint64_t n = static_cast<uint64_t>(a.n);
    for (int L = 0; L < levels; ++L) {
        a.level = L;
        if (!a.ways && !a.inplace) {
            // this level's tiles, and the tiles its completion gives the
            // children (the tail takes the default tiles)
            a.tile_keys = tile_keys_of(L);
            a.next_tile_keys = tile_keys_of(L + 1);
        }
        const uint64_t sb = seg_bound(a, L);
        const uint64_t sb_prev = L ? seg_bound(a, L - 1) : 0;
        // equal runs written at level L: at most one chunk per kFillChunk
        // keys plus one per run (the previous level's segments)
        const uint64_t fill_units = L && !a.inplace ? n / kFillChunk + sb_prev * (a.ways ? 15 : 1) : 0;
        // small segments sorted at level L: the inputs (level 0) or the
        // previous level's children
        const uint64_t small_items = L ? sb_prev * (a.ways ? 16 : 2) : std::max<uint64_t>(a.k, 1);
        if (tm) tm->start_aux();
        // (two-way plan: about 64 tile descriptors per workgroup on the
        // first levels, whose few segments have many tiles each)
        const uint64_t plan_wgs = std::max<uint64_t>(std::max<uint64_t>((sb + 3) / 4, fill_units),
                                                     a.ways ? 0 : tile_bound(a, L) / 64);
        (a.ways ? o->plan_multi : o->plan)(a, clamp_grid(plan_wgs, 2048), s);
        if (a.ways) o->map(a, clamp_grid((tile_bound(a, L) + 255) / 256, 4096), s);
        if (tm) tm->stop_aux(0, L);
        if (tm) tm->start_aux();
        o->small(a, clamp_grid(small_items, 2048), s);
        if (tm) tm->stop_aux(1, L);
        const uint64_t tb = tile_bound(a, L);
        if (tb > 0x7fffffffull) return BQS_EINVAL;
        const int tg = clamp_grid(tb, 0x7fffffff);
        if (tm) tm->start();
        if (a.inplace) {
            // (the per-tile kernels loop over the level's tiles)
            o->ip_count(a, clamp_grid(tb, 32768), s);
            o->ip_scan(a, clamp_grid(sb, 2048), s);
            o->ip_exchange(a, clamp_grid(tb, 8192), s);
            if (tm) tm->stop(2, L);
            if (tm) tm->start_aux();
            o->ip_complete(a, clamp_grid((sb + 255) / 256, 1024), s);
            if (tm) tm->stop_aux(0, L);
        } else if (a.ways) {
            o->mcount(a, tg, s);
            o->mscan(a, clamp_grid((sb + 3) / 4, 1024), s);
            o->mscatter(a, tg, s);
            if (tm) tm->stop(2, L);
        } else {
            const auto tile = a.tile_keys == o->half_tile_keys     ? o->tile_half
                              : a.tile_keys == o->double_tile_keys ? o->tile_double
                                                                   : o->tile;
            tile(a, tg, s);
            if (tm) tm->stop(2, L);
            if (tm) tm->start_aux();
            o->complete(a, clamp_grid((sb + 255) / 256, 1024), s);
            if (tm) tm->stop_aux(0, L);
        }
    }
    // whatever recursion is left: one workgroup, two-way levels with the
    // two-way tile (segments listed by multiway levels are re-tiled first)
    Args t = a;
    t.level = levels;
    t.ways = 0;
    if (!a.inplace) {
        t.tile_keys = o->tile_keys;
        t.next_tile_keys = o->tile_keys;
        t.retile = a.next_tile_keys != o->tile_keys ? 1 : 0;
    }
    if (tm) tm->start_aux();
    if (a.inplace) o->ip_tail(t, s);
    else o->tail(t, s);
    if (tm) tm->stop_aux(0, levels);
    return hipGetLastError() == hipSuccess ? BQS_OK : BQS_EHIP;
}

void drop_graph(bqs_ctx* ctx) {
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph_obj) (void)hipGraphDestroy(ctx->graph_obj);
    ctx->gexec = nullptr;
    ctx->graph_obj = nullptr;
    ctx->gkey.clear();
    ctx->glevels = 0;
}

bqs_status capture_graph(bqs_ctx* ctx, const Ops* o, const Args& a, bool segmented, int dtype, int levels) {
    drop_graph(ctx);
    if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return BQS_EHIP;
    const hipStream_t cs = ctx->cap_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return BQS_EHIP;
    const bqs_status st = enqueue_levels(o, a, segmented, ctx->check_nan != 0, dtype, levels, cs, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (st != BQS_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return st != BQS_OK ? st : BQS_EHIP;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return BQS_EHIP;
    }
    ctx->graph_obj = g;
    ctx->gexec = ex;
    ctx->glevels = levels;
    return BQS_OK;
}

// Asynchronous sort (default mode, also graph mode): enqueue and return.
bqs_status run_async(bqs_ctx* ctx, const Ops* o, Args& a, bool segmented, int dtype) {
    const hipStream_t s = ctx->stream;
    harvest(ctx, false);
    const uint64_t call = ++ctx->calls;
    const std::vector<uint64_t> shape = call_shape(o, a, segmented);
    const int levels = levels_to_enqueue(ctx, a, shape);
    bqs_stats host{};
    host.tile_keys = a.tile_keys;
    host.small_cutoff = a.small_cut;
    bqs_status st;
    if (ctx->graph) {
        const std::vector<uint64_t> key = graph_key(o, a, segmented, ctx->check_nan != 0);
        // (re)capture for a new shape, or when the depth the graph holds is
        // short of or far past what the shape needs
        if (!ctx->gexec || key != ctx->gkey || ctx->glevels < levels || ctx->glevels > levels + 4) {
            if ((st = capture_graph(ctx, o, a, segmented, dtype, levels)) != BQS_OK) return st;
            ctx->gkey = key;
        }
        if (hipGraphLaunch(ctx->gexec, s) != hipSuccess) return BQS_EHIP;
        host.graph_launches = 1;
        host.partition_launches = ctx->glevels;
        host.small_launches = ctx->glevels;
    } else {
        Timer tm{ctx, ctx->timing != 0, ctx->timing == 1, call, s};
        if ((st = enqueue_levels(o, a, segmented, ctx->check_nan != 0, dtype, levels, s, &tm)) != BQS_OK) return st;
        host.partition_launches = levels;
        host.small_launches = levels;
    }
    return record_completion(ctx, a, s, call, shape, host);
}

// ------------------------------------------------------ host-driven mode --

bqs_status ensure_pinned(bqs_ctx* ctx) {
    if (!ctx->pinned) {
        void* p = nullptr;
        if (hipHostMalloc(&p, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return BQS_EHIP;
        ctx->pinned = static_cast<Ctl*>(p);
    }
    return BQS_OK;
}

// Copies the device control block to pinned host memory and waits.
bqs_status read_ctl(bqs_ctx* ctx, const Ctl* dev) {
    if (hipMemcpyAsync(ctx->pinned, dev, kCtlHostBytes, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
        return BQS_EHIP;
    return hip_ok(hipStreamSynchronize(ctx->stream));
}

// Levels driven from the host (BQS_MODE_LEVELS): each level's counts are
// read back before its launches are sized, so every launch covers exactly
// its level's work and the call returns when the sort has finished.
bqs_status run_levels(bqs_ctx* ctx, const Ops* o, Args& a, bool segmented, int dtype) {
    harvest(ctx, true);
    bqs_status st = ensure_pinned(ctx);
    if (st != BQS_OK) return st;
    const hipStream_t s = ctx->stream;
    const uint64_t call = ++ctx->calls;
    Timer tm{ctx, ctx->timing != 0, ctx->timing == 1, call, s};
    bqs_stats stats{};
    stats.tile_keys = a.tile_keys;
    stats.small_cutoff = a.small_cut;
    std::vector<int64_t> lkeys;

    if (segmented) launch_init_segments(a, s);
    else launch_init_single(a, s);
    if (ctx->check_nan && (dtype == BQS_F32 || dtype == BQS_F64))
        hipLaunchKernelGGL(k_check_nan, dim3(clamp_grid((a.n + 255) / 256, 2048)), dim3(256), 0, s, a.x_keys, a.n,
                           dtype == BQS_F64 ? 1 : 0, a.ctl);
    if (hipGetLastError() != hipSuccess) return BQS_EHIP;
    if ((st = read_ctl(ctx, a.ctl)) != BQS_OK) return st;
    if (ctx->pinned->error) return status_of_device_error(ctx->pinned->error);
    LevelCtr cur = ctx->pinned->lc[0];
    const int cap = level_cap(a);
    for (int L = 0;; ++L) {
        a.level = L;
        const uint32_t nseg = static_cast<uint32_t>(cur.segs);
        const uint32_t ntile = static_cast<uint32_t>(cur.segs >> 32);
        const uint32_t nchunk = static_cast<uint32_t>(cur.fills >> 32);
        tm.start_aux();
        // plan: one wave per segment (4 per workgroup), one workgroup per
        // fill chunk (the two-way plan also writes the tile descriptors; the
        // multiway levels map tiles to segments in a launch of their own)
        const uint64_t plan_wgs = std::max<uint64_t>(std::max<uint64_t>((nseg + 3) / 4, nchunk),
                                                     a.ways ? 0 : ntile / 64);
        (a.ways ? o->plan_multi : o->plan)(a, clamp_grid(plan_wgs, 16384), s);
        if (nseg && a.ways) o->map(a, clamp_grid((ntile + 255) / 256, 4096), s);
        tm.stop_aux(0, L);
        uint32_t nsmall = 0;
        for (int cls = 0; cls < kSmallClasses; ++cls) nsmall += cur.smalls[cls];
        if (nsmall) {
            tm.start_aux();
            o->small(a, clamp_grid(nsmall, 16384), s);
            tm.stop_aux(1, L);
            stats.small_launches++;
        }
        if (hipGetLastError() != hipSuccess) return BQS_EHIP;
        if (nseg == 0) break;
        if (L >= cap) return BQS_EOVERFLOW;
        lkeys.push_back(static_cast<int64_t>(cur.keys));
        tm.start();
        if (a.inplace) {
            o->ip_count(a, clamp_grid(ntile, 32768), s);
            o->ip_scan(a, clamp_grid(nseg, 16384), s);
            o->ip_exchange(a, clamp_grid(ntile, 8192), s);
            tm.stop(2, L);
            tm.start_aux();
            o->ip_complete(a, clamp_grid((nseg + 255) / 256, 4096), s);
            tm.stop_aux(0, L);
        } else if (a.ways) {
            o->mcount(a, static_cast<int>(ntile), s);
            o->mscan(a, clamp_grid((nseg + 3) / 4, 4096), s);
            o->mscatter(a, static_cast<int>(ntile), s);
            tm.stop(2, L);
        } else {
            o->tile(a, static_cast<int>(ntile), s);
            tm.stop(2, L);  // the partition kernel alone
            tm.start_aux();
            o->complete(a, clamp_grid((nseg + 255) / 256, 4096), s);
            tm.stop_aux(0, L);
        }
        stats.partition_launches++;
        if (hipGetLastError() != hipSuccess) return BQS_EHIP;
        if ((st = read_ctl(ctx, a.ctl)) != BQS_OK) return st;
        if (ctx->pinned->error) return status_of_device_error(ctx->pinned->error);
        cur = ctx->pinned->lc[(L + 1) & 1];
    }
    if ((st = read_ctl(ctx, a.ctl)) != BQS_OK) return st;
    if (ctx->pinned->error) return status_of_device_error(ctx->pinned->error);
    std::vector<double> lms;
    resolve_events(ctx, call, stats, lms);
    fill_stats(stats, *ctx->pinned);
    lms.resize(lkeys.size(), 0.0);
    ctx->level_keys = lkeys;
    ctx->level_ms = lms;
    ctx->stats = stats;
    return BQS_OK;
}

// ------------------------------------------------------ persistent mode --
// Init, then one cooperative launch of every workgroup the GPU holds at
// once, which runs all levels; asynchronous like the default mode.
bqs_status run_persist(bqs_ctx* ctx, const Ops* o, Args& a, bool segmented, int dtype) {
    if (a.ways || a.inplace) return BQS_EINVAL;  // the multiway and in-place steps have no persistent form
    harvest(ctx, false);
    const hipStream_t s = ctx->stream;
    if (ctx->persist_grid <= 0 || ctx->persist_ops != o) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess) return BQS_EHIP;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return BQS_EHIP;
        const int per = o->persist_blocks_per_cu();
        if (per <= 0 || cus <= 0) return BQS_EHIP;
        ctx->persist_grid = static_cast<int64_t>(per) * cus;
        ctx->persist_ops = o;
    }
    const int grid = static_cast<int>(ctx->grid > 0 ? std::min<int64_t>(ctx->grid, ctx->persist_grid)
                                                    : ctx->persist_grid);
    const uint64_t call = ++ctx->calls;
    Timer tm{ctx, ctx->timing != 0, ctx->timing == 1, call, s};
    a.prof = 0;
    a.level = 0;
    a.retile = 0;
    if (segmented) launch_init_segments(a, s);
    else launch_init_single(a, s);
    if (ctx->check_nan && (dtype == BQS_F32 || dtype == BQS_F64))
        hipLaunchKernelGGL(k_check_nan, dim3(clamp_grid((a.n + 255) / 256, 2048)), dim3(256), 0, s, a.x_keys, a.n,
                           dtype == BQS_F64 ? 1 : 0, a.ctl);
    tm.start();
    const hipError_t e = o->persist(a, grid, s);
    tm.stop(2, -1);
    if (e != hipSuccess || hipGetLastError() != hipSuccess) return BQS_EHIP;
    bqs_stats host{};
    host.tile_keys = a.tile_keys;
    host.small_cutoff = a.small_cut;
    host.partition_launches = 1;
    return record_completion(ctx, a, s, call, call_shape(o, a, segmented), host);
}

// The entry points' common driver.
bqs_status run_sort(bqs_ctx* ctx, const Ops* o, Args& a, bool segmented, int dtype) {
    if (ctx->mode == BQS_MODE_PERSISTENT) return run_persist(ctx, o, a, segmented, dtype);
    if (ctx->mode == BQS_MODE_LEVELS) return run_levels(ctx, o, a, segmented, dtype);
    return run_async(ctx, o, a, segmented, dtype);
}

// Lays the call's buffers out in workspace [ws, ws + ws_bytes) and fills
// the kernel arguments; `ctx` supplies the parameters (null: the library's
// defaults).
bqs_status prepare_in(const bqs_ctx* ctx, void* ws, size_t ws_bytes, const Ops* o, int64_t n, int dtype, int vb,
                      int64_t k, void* keys, void* vals, Args& a) {
    const size_t kb = key_bytes(dtype);
    const int64_t S = eff_small_cut(ctx, o);
    const bool inplace = ctx && ctx->inplace;
    const bool multiway = ctx && ctx->multiway && o->mscan && !inplace;
    const Layout L = make_layout(n, kb, static_cast<size_t>(vb), k, layout_tile_keys(ctx, o), S, multiway, inplace);
    if (L.cap_tile > 0xffffffffull || L.cap_seg > 0xffffffffull || L.cap_small > 0xffffffffull ||
        L.cap_tab > 0xffffffffull)
        return BQS_EINVAL;
    if (!ws || ws_bytes < L.total) return BQS_EINVAL;
    if (overlaps(keys, static_cast<size_t>(n) * kb, ws, ws_bytes)) return BQS_EINVAL;
    if (vals && (overlaps(vals, static_cast<size_t>(n) * vb, ws, ws_bytes) ||
                 overlaps(vals, static_cast<size_t>(n) * vb, keys, static_cast<size_t>(n) * kb)))
        return BQS_EINVAL;
    char* w = static_cast<char*>(ws);
    a = Args{};
    a.ctl = reinterpret_cast<Ctl*>(w + L.ctl);
    a.x_keys = keys;
    a.x_vals = vals;
    if (inplace) {
        // every level reads and writes the caller's buffers
        a.y_keys = keys;
        a.y_vals = vals;
        a.side = nullptr;
        a.ipmask = reinterpret_cast<uint64_t*>(w + L.ipmask);
        a.iptile = reinterpret_cast<IpTile*>(w + L.iptile);
        a.iprank = reinterpret_cast<uint32_t*>(w + L.iprank);
        a.cap_tab = static_cast<uint32_t>(L.cap_tab);
        a.inplace = 1;
    } else {
        a.y_keys = w + L.yk;
        a.y_vals = vb ? w + L.yv : nullptr;
        a.side = vb ? w + L.side : nullptr;
    }
    for (int s = 0; s < 2; ++s) {
        a.segs[s] = reinterpret_cast<SegDesc*>(w + L.segs[s]);
        a.smalls[s] = reinterpret_cast<SmallItem*>(w + L.smalls[s]);
        a.fills[s] = reinterpret_cast<FillItem*>(w + L.fills[s]);
    }
    a.tile_desc = reinterpret_cast<TileDesc*>(w + L.tile_desc);
    for (int s = 0; s < 2; ++s) a.splitters[s] = reinterpret_cast<uint64_t*>(w + L.splitters[s]);
    a.toff = reinterpret_cast<uint32_t*>(w + L.toff);
    a.bcur = reinterpret_cast<uint32_t*>(w + L.bcur);
    a.bstart = reinterpret_cast<uint32_t*>(w + L.bstart);
    a.status = reinterpret_cast<unsigned long long*>(w + L.status);
    a.cap_seg = static_cast<uint32_t>(L.cap_seg);
    a.cap_tile = static_cast<uint32_t>(L.cap_tile);
    a.cap_small = static_cast<uint32_t>(L.cap_small);
    a.cap_fill = static_cast<uint32_t>(L.cap_fill);
    a.n = n;
    a.k = k;
    a.small_cut = static_cast<int>(S);
    // default sample: 127 keys for one pivot, 255 for the multiway splitters
    // (measured on 2^28 uniform int32 keys)
    const int64_t smax = ctx ? ctx->sample_max : 0;
    a.sample_max = static_cast<int>(smax > 0 ? std::min<int64_t>(smax, kMaxSample) : (multiway ? kMaxSample : 127));
    a.pivot_mode = ctx ? static_cast<int>(ctx->pivot_mode) : 0;
    a.pivot_skew = ctx ? static_cast<int>(ctx->pivot_skew) : 0;
    a.depth_limit = ctx && ctx->depth_limit > 0 ? static_cast<int>(std::min<int64_t>(ctx->depth_limit, 1 << 20))
                                                : static_cast<int>(2 * floor_log2(std::max<int64_t>(n, 2)) + 3);
    a.shuffle = ctx && ctx->shuffle ? 1 : 0;
    if (ctx && ctx->list_cap > 0) {
        // smaller lists inside the same layout: a recursion that needs more
        // room latches an overflow
        const uint32_t c = static_cast<uint32_t>(std::min<int64_t>(ctx->list_cap, 0x7fffffff));
        a.cap_seg = std::min(a.cap_seg, c);
        a.cap_small = std::min(a.cap_small, c);
        a.cap_fill = std::min(a.cap_fill, c);
    }
    a.tile_keys = static_cast<int>(eff_tile_keys(ctx, o));
    a.next_tile_keys = a.tile_keys;
    a.prof = ctx ? static_cast<int>(ctx->profile) : 0;
    a.claim = ctx && ctx->lookback ? 0 : 1;
    a.ways = multiway ? 1 : 0;
    return BQS_OK;
}

bqs_status prepare(bqs_ctx* ctx, const Ops* o, int64_t n, int dtype, int vb, int64_t k, void* keys, void* vals,
                   Args& a) {
    return prepare_in(ctx, ctx->ws, ctx->ws_bytes, o, n, dtype, vb, k, keys, vals, a);
}

// ---------------------------------------------------- no-allocation path --
// bqs_sort_noalloc's workspace: a fixed array in device memory that the
// library owns (each GPU the library runs on holds its own copy until the
// process ends).  Host code never uses the array's name as an address: the
// address of the current device's copy comes from hipGetSymbolAddress, once
// per device, and is kept in noalloc_ptr.

constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kNoAllocDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex noalloc_mu;
void* noalloc_ptr[kNoAllocDevices] = {};

// The current device's copy of the scratch array (looked up on the first
// call on that device).
bqs_status noalloc_scratch(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocDevices) return BQS_EHIP;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BQS_EHIP;
        noalloc_ptr[dev] = p;
    }
    *out = noalloc_ptr[dev];
    return BQS_OK;
}

// Writes the call's status (from the control block's error bits; none for
// a trivial call) to the caller's word.
__global__ void k_store_status(const Ctl* c, int32_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = static_cast<int32_t>(c ? status_of_device_error(c->error) : BQS_OK);
}

struct RecordKind {
    int key_dtype;  // key type of the (key, index) sort
    int words;      // 4-byte words per record
};
bool record_kind(int kind, RecordKind& rk) {
    if (kind == BQS_RECORD_VECTOR) rk = {BQS_F64, 20};
    else if (kind == BQS_RECORD_RECORD) rk = {BQS_I32, 21};
    else return false;
    return true;
}
size_t record_head(int64_t n, const RecordKind& rk) {
    return align_up(static_cast<size_t>(n) * key_bytes(rk.key_dtype)) + align_up(static_cast<size_t>(n) * 4);
}
// A call's own status is returned, not latched: the latch holds what the
// device found after the call returned.
bqs_status finish(bqs_ctx* ctx, bqs_status st) {
    (void)ctx;
    return st;
}

}  // namespace

extern "C" {

bqs_status bqs_ctx_create(bqs_ctx** out) {
    if (!out) return BQS_EINVAL;
    *out = new (std::nothrow) bqs_ctx();
    return *out ? BQS_OK : BQS_ENOMEM;
}

void bqs_ctx_destroy(bqs_ctx* ctx) {
    if (!ctx) return;
    harvest(ctx, true);  // the calls still in flight finish first
    drop_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (Ctl* p : ctx->free_slots) (void)hipHostFree(p);
    for (auto& p : ctx->pending) {
        ctx->ev_pool.push_back(p.a);
        ctx->ev_pool.push_back(p.b);
    }
    for (hipEvent_t e : ctx->ev_pool)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

bqs_status bqs_ctx_set_stream(bqs_ctx* ctx, void* hip_stream) {
    if (!ctx) return BQS_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return BQS_OK;
}

bqs_status bqs_ctx_set_workspace(bqs_ctx* ctx, void* dev_ptr, size_t bytes) {
    if (!ctx || (bytes && !dev_ptr)) return BQS_EINVAL;
    ctx->ws = dev_ptr;
    ctx->ws_bytes = bytes;
    return BQS_OK;
}

bqs_status bqs_ctx_set_param(bqs_ctx* ctx, int param, int64_t value) {
    if (!ctx) return BQS_EINVAL;
    if (value < 0) value = 0;
    switch (param) {
        case BQS_PARAM_SMALL_CUTOFF: ctx->small_cut = value; break;
        case BQS_PARAM_SAMPLE_MAX: ctx->sample_max = value; break;
        case BQS_PARAM_PIVOT_MODE:
            if (value != 0 && value != 1 && value != 3 && value != 5 && value != 23 && value != 33 &&
                value != 35 && value != 55)
                return BQS_EINVAL;
            ctx->pivot_mode = value;
            break;
        case BQS_PARAM_PIVOT_SKEW:
            if (value == 1 || value > 64) return BQS_EINVAL;
            ctx->pivot_skew = value;
            break;
        case BQS_PARAM_TIMING:
            if (value > 2) return BQS_EINVAL;
            ctx->timing = value;
            break;
        case BQS_PARAM_TILE_EPT:
            if (value != 0 && value != 8 && value != 16 && value != 32) return BQS_EINVAL;
            ctx->ept = value;
            break;
        case BQS_PARAM_GRID: ctx->grid = value; break;
        case BQS_PARAM_PROFILE: ctx->profile = value ? 1 : 0; break;
        case BQS_PARAM_GRAPH:
            ctx->graph = value ? 1 : 0;
            drop_graph(ctx);
            break;
        case BQS_PARAM_LOOKBACK: ctx->lookback = value ? 1 : 0; break;
        case BQS_PARAM_MULTIWAY: ctx->multiway = value ? 1 : 0; break;
        case BQS_PARAM_INPLACE: ctx->inplace = value ? 1 : 0; break;
        case BQS_PARAM_CHECK_NAN: ctx->check_nan = value ? 1 : 0; break;
        case BQS_PARAM_ENQUEUE_LEVELS:
            ctx->enqueue_levels = value;
            drop_graph(ctx);
            break;
        case BQS_PARAM_DEPTH_LIMIT:
            ctx->depth_limit = value;
            drop_graph(ctx);
            break;
        case BQS_PARAM_LIST_CAP:
            ctx->list_cap = value;
            drop_graph(ctx);
            break;
        case BQS_PARAM_SHUFFLE:
            ctx->shuffle = value ? 1 : 0;
            drop_graph(ctx);
            break;
        case BQS_PARAM_MODE:
            if (value != BQS_MODE_ASYNC && value != BQS_MODE_LEVELS && value != BQS_MODE_PERSISTENT)
                return BQS_EINVAL;
            ctx->mode = value;
            drop_graph(ctx);
            break;
        default: return BQS_EINVAL;
    }
    return BQS_OK;
}

int64_t bqs_ctx_get_param(const bqs_ctx* ctx, int param) {
    if (!ctx) return -1;
    switch (param) {
        case BQS_PARAM_SMALL_CUTOFF: return ctx->small_cut;
        case BQS_PARAM_SAMPLE_MAX: return ctx->sample_max;
        case BQS_PARAM_PIVOT_MODE: return ctx->pivot_mode;
        case BQS_PARAM_PIVOT_SKEW: return ctx->pivot_skew;
        case BQS_PARAM_TIMING: return ctx->timing;
        case BQS_PARAM_TILE_EPT: return ctx->ept;
        case BQS_PARAM_GRID: return ctx->grid;
        case BQS_PARAM_PROFILE: return ctx->profile;
        case BQS_PARAM_MODE: return ctx->mode;
        case BQS_PARAM_GRAPH: return ctx->graph;
        case BQS_PARAM_LOOKBACK: return ctx->lookback;
        case BQS_PARAM_MULTIWAY: return ctx->multiway;
        case BQS_PARAM_INPLACE: return ctx->inplace;
        case BQS_PARAM_CHECK_NAN: return ctx->check_nan;
        case BQS_PARAM_ENQUEUE_LEVELS: return ctx->enqueue_levels;
        case BQS_PARAM_DEPTH_LIMIT: return ctx->depth_limit;
        case BQS_PARAM_LIST_CAP: return ctx->list_cap;
        case BQS_PARAM_SHUFFLE: return ctx->shuffle;
        default: return -1;
    }
}

bqs_status bqs_ctx_get_stats(bqs_ctx* ctx, bqs_stats* out) {
    if (!ctx || !out) return BQS_EINVAL;
    harvest(ctx, true);
    *out = ctx->stats;
    return BQS_OK;
}

bqs_status bqs_ctx_get_level(bqs_ctx* ctx, int level, int64_t* keys, double* partition_ms) {
    if (!ctx) return BQS_EINVAL;
    harvest(ctx, true);
    if (level < 0 || static_cast<size_t>(level) >= ctx->level_keys.size()) return BQS_EINVAL;
    if (keys) *keys = ctx->level_keys[level];
    if (partition_ms) *partition_ms = ctx->level_ms[level];
    return BQS_OK;
}

size_t bqs_workspace_bytes(const bqs_ctx* ctx, int64_t n_total, bqs_dtype key, int32_t val_bytes,
                           int64_t k_segments) {
    if (n_total < 0 || k_segments < 0) return 0;
    const Ops* o = select_ops(ctx, key, val_bytes);
    if (!o) return 0;
    const Layout L = make_layout(n_total, key_bytes(key), static_cast<size_t>(val_bytes),
                                 std::max<int64_t>(k_segments, 1), layout_tile_keys(ctx, o), eff_small_cut(ctx, o),
                                 ctx && ctx->multiway && o->mscan && !ctx->inplace, ctx && ctx->inplace);
    return L.total;
}

bqs_status bqs_sort(void* keys, int64_t n, bqs_dtype dtype, bqs_ctx* ctx) {
    if (!ctx || n < 0 || (n > 0 && !keys)) return BQS_EINVAL;
    const Ops* o = select_ops(ctx, dtype, 0);
    if (!o) return BQS_EDTYPE;
    if (n <= 1) return BQS_OK;
    if (n >= (int64_t(1) << 31)) return BQS_EINVAL;
    Args a;
    bqs_status st = prepare(ctx, o, n, dtype, 0, 1, keys, nullptr, a);
    if (st != BQS_OK) return st;
    return finish(ctx, run_sort(ctx, o, a, false, dtype));
}

bqs_status bqs_sort_pairs(void* keys, void* vals, int64_t n, bqs_dtype key, int32_t val_bytes,
                          bqs_ctx* ctx) {
    if (!ctx || n < 0 || (n > 0 && (!keys || !vals))) return BQS_EINVAL;
    if (val_bytes != 4 && val_bytes != 8) return BQS_EDTYPE;
    const Ops* o = select_ops(ctx, key, val_bytes);
    if (!o) return BQS_EDTYPE;
    if (n <= 1) return BQS_OK;
    if (n >= (int64_t(1) << 31)) return BQS_EINVAL;
    Args a;
    bqs_status st = prepare(ctx, o, n, key, val_bytes, 1, keys, vals, a);
    if (st != BQS_OK) return st;
    return finish(ctx, run_sort(ctx, o, a, false, key));
}

bqs_status bqs_sort_segments(void* keys, const int64_t* offsets, int64_t k, int64_t n_total,
                             bqs_dtype dtype, bqs_ctx* ctx) {
    if (!ctx || k < 0 || n_total < 0 || (n_total > 0 && !keys) || (k > 0 && !offsets)) return BQS_EINVAL;
    const Ops* o = select_ops(ctx, dtype, 0);
    if (!o) return BQS_EDTYPE;
    if (k == 0 || n_total <= 1) return BQS_OK;
    if (ctx->ticks && ctx->ticks_count < k + 1) return BQS_EINVAL;
    Args a;
    bqs_status st = prepare(ctx, o, n_total, dtype, 0, k, keys, nullptr, a);
    if (st != BQS_OK) return st;
    a.offsets = offsets;
    a.ticks = ctx->ticks;
    return finish(ctx, run_sort(ctx, o, a, true, dtype));
}

bqs_status bqs_sort_segments_pairs(void* keys, void* vals, const int64_t* offsets, int64_t k,
                                   int64_t n_total, bqs_dtype key, int32_t val_bytes, bqs_ctx* ctx) {
    if (!ctx || k < 0 || n_total < 0 || (n_total > 0 && (!keys || !vals)) || (k > 0 && !offsets))
        return BQS_EINVAL;
    if (val_bytes != 4 && val_bytes != 8) return BQS_EDTYPE;
    const Ops* o = select_ops(ctx, key, val_bytes);
    if (!o) return BQS_EDTYPE;
    if (k == 0 || n_total <= 1) return BQS_OK;
    if (ctx->ticks && ctx->ticks_count < k + 1) return BQS_EINVAL;
    Args a;
    bqs_status st = prepare(ctx, o, n_total, key, val_bytes, k, keys, vals, a);
    if (st != BQS_OK) return st;
    a.offsets = offsets;
    a.ticks = ctx->ticks;
    return finish(ctx, run_sort(ctx, o, a, true, key));
}

bqs_status bqs_sort_noalloc(void* keys, int64_t n, bqs_dtype dtype, void* hip_stream, int32_t* status_out) {
    if (n < 0 || (n > 0 && !keys)) return BQS_EINVAL;
    const Ops* o = select_ops(nullptr, dtype, 0);
    if (!o) return BQS_EDTYPE;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (n <= 1) {
        if (status_out) hipLaunchKernelGGL(k_store_status, dim3(1), dim3(64), 0, s, nullptr, status_out);
        return hipGetLastError() == hipSuccess ? BQS_OK : BQS_EHIP;
    }
    if (n >= (int64_t(1) << 31)) return BQS_EINVAL;
    if (bqs_workspace_bytes(nullptr, n, dtype, 0, 1) > kNoAllocBytes) return BQS_ETOOBIG;
    void* ws = nullptr;
    bqs_status st = noalloc_scratch(&ws);
    if (st != BQS_OK) return st;
    Args a;
    if ((st = prepare_in(nullptr, ws, kNoAllocBytes, o, n, dtype, 0, 1, keys, nullptr, a)) != BQS_OK) return st;
    if ((st = enqueue_levels(o, a, false, false, dtype, estimate_levels(a), s, nullptr)) != BQS_OK) return st;
    if (status_out) hipLaunchKernelGGL(k_store_status, dim3(1), dim3(64), 0, s, a.ctl, status_out);
    return hipGetLastError() == hipSuccess ? BQS_OK : BQS_EHIP;
}

// ------------------------------------------------------------- records --

size_t bqs_records_workspace_bytes(const bqs_ctx* ctx, int64_t n, int kind) {
    RecordKind rk;
    if (n < 0 || !record_kind(kind, rk)) return 0;
    return record_head(n, rk) + bqs_workspace_bytes(ctx, std::max<int64_t>(n, 2), static_cast<bqs_dtype>(rk.key_dtype),
                                                    4, 1);
}

bqs_status bqs_sort_records(const void* in, void* out, int64_t n, int kind, bqs_ctx* ctx) {
    RecordKind rk;
    if (!ctx || n < 0 || (n > 0 && (!in || !out))) return BQS_EINVAL;
    if (!record_kind(kind, rk)) return BQS_EDTYPE;
    if (n >= (int64_t(1) << 31)) return BQS_EINVAL;
    const size_t rec = static_cast<size_t>(rk.words) * 4;
    if (overlaps(in, n * rec, out, n * rec) || overlaps(in, n * rec, ctx->ws, ctx->ws_bytes) ||
        overlaps(out, n * rec, ctx->ws, ctx->ws_bytes))
        return BQS_EINVAL;
    if (n == 0) return BQS_OK;
    const size_t head = record_head(n, rk);
    if (!ctx->ws || ctx->ws_bytes < bqs_records_workspace_bytes(ctx, n, kind)) return BQS_EINVAL;
    char* w = static_cast<char*>(ctx->ws);
    void* keys = w;
    uint32_t* idx = reinterpret_cast<uint32_t*>(w + align_up(static_cast<size_t>(n) * key_bytes(rk.key_dtype)));
    const hipStream_t s = ctx->stream;
    const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
    if (kind == BQS_RECORD_VECTOR)
        hipLaunchKernelGGL(k_vector_keys, dim3(blocks), dim3(256), 0, s, static_cast<const double*>(in), n,
                           static_cast<double*>(keys), idx);
    else
        hipLaunchKernelGGL(k_record_keys, dim3(blocks), dim3(256), 0, s, static_cast<const int32_t*>(in), n,
                           static_cast<int32_t*>(keys), idx);
    if (hipGetLastError() != hipSuccess) return finish(ctx, BQS_EHIP);
    bqs_status st = BQS_OK;
    if (n > 1) {
        // the (key, index) sort runs in the rest of the workspace, host-driven
        const Ops* o = select_ops(ctx, rk.key_dtype, 4);
        if (!o) return BQS_EDTYPE;
        void* ws0 = ctx->ws;
        const size_t wb0 = ctx->ws_bytes;
        const int64_t graph0 = ctx->graph;
        ctx->ws = w + head;
        ctx->ws_bytes = wb0 - head;
        ctx->graph = 0;
        Args a;
        st = prepare(ctx, o, n, rk.key_dtype, 4, 1, keys, idx, a);
        if (st == BQS_OK) st = run_sort(ctx, o, a, false, rk.key_dtype);
        ctx->ws = ws0;
        ctx->ws_bytes = wb0;
        ctx->graph = graph0;
        if (st != BQS_OK) return finish(ctx, st);
    }
    const int64_t words = n * rk.words;
    const unsigned gblocks = static_cast<unsigned>(std::min<int64_t>((words + 255) / 256, 65536));
    hipLaunchKernelGGL(k_gather_words, dim3(gblocks), dim3(256), 0, s, static_cast<const uint32_t*>(in), idx, n,
                       rk.words, static_cast<uint32_t*>(out));
    if (hipGetLastError() != hipSuccess) return finish(ctx, BQS_EHIP);
    return BQS_OK;
}

bqs_status bqs_ctx_sync_status(bqs_ctx* ctx) {
    if (!ctx) return BQS_EINVAL;
    harvest(ctx, true);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) latch(ctx, BQS_EHIP);
    const bqs_status st = ctx->latched;
    ctx->latched = BQS_OK;
    return st;
}

bqs_status bqs_ctx_set_segment_ticks(bqs_ctx* ctx, uint64_t* ticks, int64_t count) {
    if (!ctx || (ticks && count < 1)) return BQS_EINVAL;
    ctx->ticks = reinterpret_cast<unsigned long long*>(ticks);
    ctx->ticks_count = ticks ? count : 0;
    drop_graph(ctx);
    return BQS_OK;
}

bqs_status bqs_ctx_poll_status(bqs_ctx* ctx) {
    if (!ctx) return BQS_EINVAL;
    harvest(ctx, false);
    const bqs_status st = ctx->latched;
    ctx->latched = BQS_OK;
    return st;
}

const char* bqs_status_str(bqs_status s) {
    switch (s) {
        case BQS_OK: return "ok";
        case BQS_EINVAL: return "invalid argument";
        case BQS_EDTYPE: return "unsupported dtype";
        case BQS_ENOMEM: return "out of host memory";
        case BQS_EHIP: return "HIP runtime error";
        case BQS_ENAN: return "NaN key";
        case BQS_EOVERFLOW: return "device work list overflow";
        case BQS_ETOOBIG: return "input larger than the no-allocation scratch";
        default: return "unknown status";
    }
}

int bqs_version(void) { return 200; }

}  // extern "C"
