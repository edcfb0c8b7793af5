// Internal interface between the host runtime (bqs_api.hip) and the kernel
// translation units.  Not part of the public ABI (include/bqs.h).
//
// Work is organised by recursion level L (Quicksort, Algorithm 1, unrolled
// breadth first).  Level L reads its segments from buffer (L & 1) -- 0 is the
// caller's array X, 1 the workspace copy Y -- and writes the partitioned
// result to buffer ((L + 1) & 1).  Every list that level L consumes lives in
// slot (L & 1) and is produced by level L-1 (or by the init kernels for L=0):
//   segs   : segments partitioned at level L (more than small_cut keys)
//   smalls : segments finished at level L by the in-LDS sort
//   fills  : runs of keys equal to a level L-1 pivot, written at level L
// The kernels of one level, in stream order: plan (pivots, tile map, fills),
// small (in-LDS sorts), partition (tiles; appends the level L+1 lists).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bqs.h"
#define BQS_STATUS_MAP_FN __host__ __device__ inline
#include "bqs_status_map.h"

namespace bqs {

constexpr int kFillChunk = 4096;  // keys per fill work unit
constexpr int kSmallClasses = 9;  // small-sort size classes: segments of at most 64 << c keys

// Size class of a small segment of m >= 1 keys: the smallest c with
// m <= 64 << c.
__host__ __device__ inline int small_class(int64_t m) {
    int c = 0;
    while ((int64_t(64) << c) < m) ++c;
    return c;
}
constexpr int kMaxSample = 255;   // largest pivot sample

// Tiles of a segment [lo, hi) of a partition level with T keys per tile:
// tile j covers [lo + j*T, min(lo + (j+1)*T, hi)), so only a segment's last
// tile is partial.
__host__ __device__ inline uint32_t seg_tiles(int64_t lo, int64_t hi, int64_t T) {
    return static_cast<uint32_t>((hi - lo + T - 1) / T);
}

struct SegDesc {
    int64_t lo, hi;      // [lo, hi) in the level's source buffer
    uint64_t pivot;      // pivot as an order key (set by the plan kernel)
    uint64_t pivot_raw;  // pivot as stored bits
    uint32_t t0, nt;     // tiles [t0, t0 + nt) of this level belong to the segment
    uint32_t depth;
    uint32_t pad;        // multiway levels: splitters in use; in-place levels: kSegForced
    // cursor claims (keys only): low 32 bits keys already placed in the left
    // run, high 32 bits in the right run (cleared by the plan kernel).
    // In-place levels: low 32 bits class-L keys, high 32 bits keys equal to
    // the pivot (written by the scan step)
    unsigned long long cursor;
    uint32_t origin;     // segmented calls: the input segment this one is part of
    uint32_t pad2;
};

// SegDesc::pad bits of the in-place step.  kSegForced: the pivot was fixed
// by the parent (the parent's pivot, the segment's smallest key) and the
// classes are x <= p, so the left part holds only keys equal to p and is
// finished.  kSegARight: the right part is the larger one, and its tiles
// own the exchange of misplaced keys.
constexpr uint32_t kSegForced = 1u;
constexpr uint32_t kSegARight = 2u;

// In-place step: tiles of kIpT keys (256 threads x 16), one bit per key.
constexpr int kIpNT = 256;
constexpr int kIpEPT = 16;
constexpr int kIpT = kIpNT * kIpEPT;
constexpr int kIpWords = kIpT / 64;  // 64-bit class words per tile

// Per tile of an in-place level: counts from the count step; misplaced
// counts, ranks and the segment's values from the scan step.  mis[0]: keys
// of the tile left of the segment's boundary that are not class L; mis[1]:
// class-L keys right of it.  rank[0]: rank of the tile's first misplaced
// key left of the boundary, counted from the segment's left end; rank[1]:
// rank of its first misplaced key right of the boundary, counted from the
// segment's right end (so its right-side keys have ranks [rank[1],
// rank[1] + mis[1]) in descending position order).
struct IpTile {
    uint32_t nl, neq;
    uint32_t mis[2];
    uint32_t rank[2];
    uint32_t seg_nl;   // the segment's class-L keys: boundary b = lo + seg_nl
    uint32_t flags;    // kSegARight: the right part's tiles own the exchange
    uint32_t tbase;    // the segment's first entry in the level's rank table
    uint32_t pad[3];
};

// Rank table of an in-place level: per segment, entry j names the tile of
// the partner side (the smaller part) that holds the misplaced key of rank
// j * kIpRankStep, so that an owning tile finds its first partner tile with
// one lookup and a short walk.
constexpr int kIpRankStep = 256;

// Per-tile copy of what a partition tile needs, written by the map kernel so
// that a tile reaches its segment with one load.
struct TileDesc {
    int64_t lo, hi;      // the tile's segment
    uint64_t pivot;      // the segment's pivot as an order key
    uint32_t t0;         // first tile of the segment
    uint32_t si;         // segment index in the level's list
};

struct SmallItem {
    int64_t lo, hi;
    uint32_t origin;  // segmented calls: the input segment this one is part of
    uint32_t pad;
};

struct FillItem {
    int64_t dst;     // first position of the equal run in X
    int64_t len;     // run length
    int64_t side;    // first position of the run's payloads in the side buffer
    uint64_t raw;    // key bits of the pivot
    uint32_t chunk0; // first fill work unit of this item
    uint32_t origin; // segmented calls: the input segment the run belongs to
    uint64_t pad1;
};

struct LevelCtr {
    unsigned long long segs;   // low 32 bits: segments, high 32 bits: tiles
    unsigned long long fills;  // low 32 bits: items, high 32 bits: work units
    unsigned int smalls[kSmallClasses];  // small segments per size class
    unsigned int tile_next;    // tile claim counter of the level that consumes this slot
    unsigned int tab;          // in-place levels: rank-table entries handed out
    unsigned long long keys;   // keys in the segments of this list (statistics)
};

constexpr int kMaxXcd = 16;  // XCD ids the persistent barrier can index (MI355X has 8)
constexpr int kLevelStats = 128;  // levels with their own statistics slot (deeper ones share the last)

__host__ __device__ inline int level_slot(int level) { return level < kLevelStats ? level : kLevelStats - 1; }

struct Ctl {
    LevelCtr lc[2];
    unsigned int error;
    unsigned int levels;  // levels that partitioned at least one segment
    unsigned long long part_keys;
    unsigned long long small_keys;
    unsigned long long fill_keys;
    unsigned long long tiles;
    // profile counters (only with Args::prof): tiles, look-back rounds,
    // look-back polls, look-back cycles, tile cycles, load+count cycles
    unsigned long long prof[8];
    // small-sort profile (only with Args::prof): segments, then cycles of
    // thread 0 per phase summed over segments (load and key range, bucket
    // counts, bucket starts, scatter, in-bucket order and store)
    unsigned long long sprof[8];
    unsigned long long level_keys[kLevelStats];  // keys partitioned per level (statistics)
    // persistent mode: grid barrier.  Global arrivals (one per XCD) and the
    // generation that waiting workgroups poll, each on a line of its own;
    // arrivals per XCD (one line each); resident workgroups per XCD.
    alignas(256) unsigned int bar_arrive;
    alignas(256) unsigned int bar_gen;
    unsigned int bar_err;  // `error` as it stood when the current barrier generation opened
    alignas(256) unsigned int xcd_arrive[kMaxXcd][64];
    unsigned int xcd_n[kMaxXcd];
};

struct Args {
    Ctl* ctl;
    void* x_keys;
    void* y_keys;
    void* x_vals;
    void* y_vals;
    void* side;
    SegDesc* segs[2];
    SmallItem* smalls[2];      // per slot: kSmallClasses regions of cap_small items
    FillItem* fills[2];
    TileDesc* tile_desc;
    unsigned long long* status;
    uint32_t cap_seg, cap_tile, cap_small, cap_fill;
    int64_t n;
    const int64_t* offsets;
    int64_t k;
    int level;
    int small_cut;
    int sample_max;
    int pivot_mode;
    int pivot_skew;  // >= 2: pivot = the sample's 1/skew quantile (skewed-pivot study)
    int depth_limit;
    int tile_keys;       // keys per tile of this level
    int next_tile_keys;  // keys per tile of the next level (the completion tiles the children)
    int prof;
    int claim;  // 1: keys-only tiles claim their ranges with the segment's cursor
    int ways;   // 1: multiway partition levels (keys only)
    int retile; // 1: the first level's segments were tiled for another tile size (tail kernel)
    int shuffle; // stress test: tiles claimed out of order within windows of 64, delayed publication
    int inplace; // 1: in-place levels (keys and payloads stay in x_keys / x_vals)
    uint64_t* ipmask;        // in-place levels: class bits, kIpWords words per tile
    IpTile* iptile;          // in-place levels: per tile counts and running sums
    uint32_t* iprank;        // in-place levels: rank table (cap_tab entries)
    uint32_t cap_tab;
    // segmented calls with a completion clock: per input segment the device
    // wall clock (100 MHz) when its last key became final, and at [k] the
    // call's start (nullptr: not recorded)
    unsigned long long* ticks;
    uint64_t* splitters[2];  // per slot: 16 order keys per segment
    uint32_t* toff;          // per tile: offset of its keys inside each bucket
    uint32_t* bcur;          // per segment: bucket cursors (stride 32)
    uint32_t* bstart;        // per segment: bucket starts from the segment start
};

struct Ops {
    int tile_keys;  // keys per partition tile
    int small_max;      // capacity of the in-LDS small sort
    int small_default;  // default cutoff (measured best for the tile size)
    void (*plan)(const Args&, int grid, hipStream_t);
    void (*map)(const Args&, int grid, hipStream_t);
    // every small segment of the level (all size classes), one per workgroup
    void (*small)(const Args&, int grid, hipStream_t);
    void (*tile)(const Args&, int grid, hipStream_t);
    // segment completion after a partition launch: children and equal runs
    // of every segment of the level
    void (*complete)(const Args&, int grid, hipStream_t);
    // multiway levels (keys only; nullptr otherwise): splitters + fills,
    // per-tile histograms, per-segment offsets + lists, per-tile scatter
    void (*plan_multi)(const Args&, int grid, hipStream_t);
    void (*mcount)(const Args&, int grid, hipStream_t);
    void (*mscan)(const Args&, int grid, hipStream_t);
    void (*mscatter)(const Args&, int grid, hipStream_t);
    // persistent mode: every level in one cooperative launch of `grid`
    // resident workgroups; small segments up to persist_small_max keys
    hipError_t (*persist)(const Args&, int grid, hipStream_t);
    // the levels from a.level on, by one workgroup (an ordinary launch): the
    // rest of a sort whose enqueued levels did not reach the end
    void (*tail)(const Args&, hipStream_t);
    int (*persist_blocks_per_cu)();
    int persist_small_max;
    int multi_tile_keys;  // keys per tile of the multiway levels (0 without them)
    // in-place levels: class bits and counts per tile, boundary and running
    // sums per segment, exchange of misplaced keys per tile, children per
    // segment; and the one-workgroup tail of an in-place sort
    void (*ip_count)(const Args&, int grid, hipStream_t);
    void (*ip_scan)(const Args&, int grid, hipStream_t);
    void (*ip_exchange)(const Args&, int grid, hipStream_t);
    void (*ip_complete)(const Args&, int grid, hipStream_t);
    void (*ip_tail)(const Args&, hipStream_t);
    // keys-only two-way levels with many segments: half-size tiles (more
    // workgroups in flight; their claims spread over many cursors), or 0
    int half_tile_keys;
    void (*tile_half)(const Args&, int grid, hipStream_t);
    // keys-only two-way levels of few, large segments: double-size tiles on
    // twice the threads (half the claims on the few cursors), or 0
    int double_tile_keys;
    void (*tile_double)(const Args&, int grid, hipStream_t);
};

// The map step of level `level`, as thread `gtid` of `gstride`: every tile
// finds its segment (the list is ordered by first tile) and gets its
// descriptor; its look-back status word is cleared.
__device__ inline void map_tiles(const Args& a, int level, uint32_t gtid, uint32_t gstride) {
    const int p = level & 1;
    const unsigned long long sc = a.ctl->lc[p].segs;
    // counts past the capacities mean an overflow was latched: only the
    // entries that were written are read
    const uint32_t nseg = static_cast<uint32_t>(sc) < a.cap_seg ? static_cast<uint32_t>(sc) : a.cap_seg;
    const uint32_t ntile = static_cast<uint32_t>(sc >> 32) < a.cap_tile ? static_cast<uint32_t>(sc >> 32) : a.cap_tile;
    const SegDesc* segs = a.segs[p];
    for (uint32_t t = gtid; t < ntile; t += gstride) {
        uint32_t lo_i = 0, hi_i = nseg;
        while (hi_i - lo_i > 1) {
            const uint32_t mid = (lo_i + hi_i) >> 1;
            if (segs[mid].t0 <= t) lo_i = mid; else hi_i = mid;
        }
        const SegDesc& sd = segs[lo_i];
        TileDesc d;
        d.lo = sd.lo;
        d.hi = sd.hi;
        d.pivot = sd.pivot;
        d.t0 = sd.t0;
        d.si = lo_i;
        a.tile_desc[t] = d;
        a.status[t] = 0;
    }
}

// Kernel tables, one per payload kind; nullptr for an unsupported request.
const Ops* ops_keys(int dtype, int ept);
const Ops* ops_pairs32(int dtype);
const Ops* ops_pairs64(int dtype);

// Dtype-independent set-up kernels (bqs_api.hip).
void launch_init_single(const Args& a, hipStream_t s);
void launch_init_segments(const Args& a, hipStream_t s);
void launch_map(const Args& a, int grid, hipStream_t s);

}  // namespace bqs
