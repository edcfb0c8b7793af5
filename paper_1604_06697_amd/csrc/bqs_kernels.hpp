// Device code of the block-partition sort for gfx950 (CDNA4, wave64).
//
// The paper's block partition (Section 3, Algorithm 3) scans a block of B
// elements, stores the comparison outcomes as offsets into a buffer (the
// counter is advanced by the Boolean result, never by a branch), and moves
// the elements in a second, comparison-free phase.  On the GPU one
// workgroup plays the role of one block, a "tile" of NT*EPT keys:
//   * scanning phase   -- every lane compares its keys with the pivot; the
//     outcomes become wave masks (ballot) whose popcounts are the per-wave
//     counts and whose masked bit counts (mbcnt) are the lane ranks;
//   * offsets          -- an LDS prefix sum over (item, wave) counts gives
//     every key its rank in its class (less / greater / equal) inside the
//     tile, i.e. the paper's offsets_L / offsets_R buffers, for all keys at
//     once;
//   * the two cursors  -- the paper's left cursor l (advancing by B) and
//     right cursor r (retreating by B) become a left and a right output
//     range per tile, claimed through a decoupled look-back over the tile
//     status words of the same segment;
//   * rearrangement    -- keys are written to LDS at their ranks and copied
//     out coalesced: the left run grows from the segment start, the right
//     run from the segment end, into the other buffer (out of place).
// Keys equal to the pivot form a third class (the paper's duplicate check,
// Section 3.2, done in one pass): they are excluded from the recursion and
// written once the segment's totals are known.

#pragma once

#include <type_traits>

#include "bqs_internal.h"

namespace bqs {

// ---------------------------------------------------------------------------
// Order transform: stored key bits -> unsigned integer whose unsigned < is
// the total order of the key type (signed ints: flip the sign bit; floats:
// IEEE-754 totalOrder, -0 < +0).  Keys move as raw bits; the transform is
// applied only where keys are compared.

template <int DT>
struct KeyT;

template <>
struct KeyT<BQS_I32> {
    using raw = uint32_t;
    __device__ static uint32_t ord(uint32_t x) { return x ^ 0x80000000u; }
    __device__ static uint32_t inv(uint32_t u) { return u ^ 0x80000000u; }
};
template <>
struct KeyT<BQS_U32> {
    using raw = uint32_t;
    __device__ static uint32_t ord(uint32_t x) { return x; }
    __device__ static uint32_t inv(uint32_t u) { return u; }
};
template <>
struct KeyT<BQS_F32> {
    using raw = uint32_t;
    __device__ static uint32_t ord(uint32_t b) {
        return b ^ (static_cast<uint32_t>(static_cast<int32_t>(b) >> 31) | 0x80000000u);
    }
    __device__ static uint32_t inv(uint32_t u) { return u ^ (((u >> 31) - 1u) | 0x80000000u); }
};
template <>
struct KeyT<BQS_I64> {
    using raw = uint64_t;
    __device__ static uint64_t ord(uint64_t x) { return x ^ 0x8000000000000000ull; }
    __device__ static uint64_t inv(uint64_t u) { return u ^ 0x8000000000000000ull; }
};
template <>
struct KeyT<BQS_U64> {
    using raw = uint64_t;
    __device__ static uint64_t ord(uint64_t x) { return x; }
    __device__ static uint64_t inv(uint64_t u) { return u; }
};
template <>
struct KeyT<BQS_F64> {
    using raw = uint64_t;
    __device__ static uint64_t ord(uint64_t b) {
        return b ^ (static_cast<uint64_t>(static_cast<int64_t>(b) >> 63) | 0x8000000000000000ull);
    }
    __device__ static uint64_t inv(uint64_t u) {
        return u ^ (((u >> 63) - 1ull) | 0x8000000000000000ull);
    }
};

struct NoVal {};

template <class V>
struct ValStore {
    using type = V;
};
template <>
struct ValStore<NoVal> {
    using type = uint32_t;  // placeholder, never read or written
};

// ---------------------------------------------------------------------------
// Wave (64-lane) helpers.

__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x & 63); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int d) {
    const int lo = __shfl_up(static_cast<int>(static_cast<uint32_t>(v)), d, 64);
    const int hi = __shfl_up(static_cast<int>(static_cast<uint32_t>(v >> 32)), d, 64);
    return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ __forceinline__ uint64_t shfl_down64(uint64_t v, int d) {
    const int lo = __shfl_down(static_cast<int>(static_cast<uint32_t>(v)), d, 64);
    const int hi = __shfl_down(static_cast<int>(static_cast<uint32_t>(v >> 32)), d, 64);
    return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int d) {
    const int lo = __shfl_xor(static_cast<int>(static_cast<uint32_t>(v)), d, 64);
    const int hi = __shfl_xor(static_cast<int>(static_cast<uint32_t>(v >> 32)), d, 64);
    return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ __forceinline__ uint64_t bcast64(uint64_t v, int src) {
    const int lo = __shfl(static_cast<int>(static_cast<uint32_t>(v)), src, 64);
    const int hi = __shfl(static_cast<int>(static_cast<uint32_t>(v >> 32)), src, 64);
    return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

template <class O>
__device__ __forceinline__ O shfl_xor_o(O v, int d) {
    if constexpr (sizeof(O) == 8) return shfl_xor64(v, d);
    else return static_cast<O>(__shfl_xor(static_cast<int>(v), d, 64));
}

// `lane` is passed in so that callers inside loops can hand over an opaque
// copy: otherwise the six lane >= d masks are hoisted out of the loop and
// held in scalar registers across it.
__device__ __forceinline__ uint64_t wave_inclusive_sum(uint64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t t = shfl_up64(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

// Value the compiler cannot see through: keeps cheap per-lane compares
// inside the loop instead of hoisting their masks into scalar registers.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += shfl_xor64(v, d);
    return v;
}

// ---------------------------------------------------------------------------
// Tile status words for the decoupled look-back: 2-bit flag, 31-bit count of
// keys < pivot (L) and 31-bit count of keys > pivot (G).  AGG: the tile's own
// counts; INC: inclusive counts of the segment's tiles 0..j.

constexpr uint64_t kStAgg = 1, kStInc = 2;
constexpr uint64_t kM31 = 0x7fffffffull;
constexpr uint64_t kM21 = 0x1fffffull;

__device__ __forceinline__ uint64_t st_pack(uint64_t flag, uint64_t l, uint64_t g) {
    return (flag << 62) | (l << 31) | g;
}

__device__ __forceinline__ uint64_t ld_status(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_status(unsigned long long* p, uint64_t v) {
    __hip_atomic_store(p, static_cast<unsigned long long>(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // 64-bit finaliser (MurmurHash3 fmix64) used to jitter sample positions
    z ^= z >> 33;
    z *= 0xff51afd7ed558ccdull;
    z ^= z >> 33;
    z *= 0xc4ceb9fe1a85ec53ull;
    z ^= z >> 33;
    return z;
}

// ---------------------------------------------------------------------------
// Completion clock of segmented calls: from now on a piece of input segment
// `origin` is final (its keys are in place in X).  The latest such time of a
// segment is its completion time.

__device__ __forceinline__ void mark_done(const Args& a, uint32_t origin) {
    if (a.ticks) atomicMax(&a.ticks[origin], static_cast<unsigned long long>(wall_clock64()));
}

// Writes the equal-key runs recorded for level p into X: keys get the stored
// bits of the run's key, pairs their payloads from the side buffer.  One
// workgroup per work unit of kFillChunk keys (all NT threads); `bid` of
// `nblk` workgroups.
template <int DT, class V, int NT>
__device__ void run_fills(const Args& a, int p, uint32_t bid, uint32_t nblk) {
    using R = typename KeyT<DT>::raw;
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    const Ctl* c = a.ctl;
    const int tid = threadIdx.x;
    const unsigned long long fc = c->lc[p].fills;
    uint32_t nfill = static_cast<uint32_t>(fc);
    if (nfill > a.cap_fill) nfill = a.cap_fill;  // an overflow was latched
    if (nfill == 0) return;
    const uint32_t nchunk = static_cast<uint32_t>(fc >> 32);
    R* xk = static_cast<R*>(a.x_keys);
    // every item has at least one chunk, so item i starts at a chunk in
    // [i, i + extra]: the item of chunk ch lies in [ch - extra, ch]
    const uint32_t extra = nchunk > nfill ? nchunk - nfill : 0u;
    for (uint32_t ch = bid; ch < nchunk; ch += nblk) {
        // items are ordered by chunk0: find the last one starting at or before ch
        uint32_t lo_i = ch > extra ? ch - extra : 0u;
        uint32_t hi_i = ch + 1 < nfill ? ch + 1 : nfill;
        while (hi_i - lo_i > 1) {
            const uint32_t mid = (lo_i + hi_i) >> 1;
            if (a.fills[p][mid].chunk0 <= ch) lo_i = mid; else hi_i = mid;
        }
        const FillItem f = a.fills[p][lo_i];
        const int64_t b = static_cast<int64_t>(ch - f.chunk0) * kFillChunk;
        const int64_t e = b + kFillChunk < f.len ? b + kFillChunk : f.len;
        const R raw = static_cast<R>(f.raw);
        for (int64_t t = b + tid; t < e; t += NT) {
            xk[f.dst + t] = raw;
            if constexpr (HV) {
                static_cast<V*>(a.x_vals)[f.dst + t] = static_cast<const V*>(a.side)[f.side + t];
            }
        }
        if (a.ticks) {
            __syncthreads();  // every thread's stores of the chunk are issued
            if (tid == 0) mark_done(a, f.origin);
        }
    }
}

// Workgroup 0 of a plan step clears the lists that level p's partition
// fills (slot q) and counts the level.
__device__ inline void reset_next_slot(Ctl* c, int q, uint32_t nseg, uint32_t bid) {
    if (bid == 0 && threadIdx.x == 0) {
        c->lc[q].segs = 0;
        c->lc[q].fills = 0;
        for (int k = 0; k < kSmallClasses; ++k) c->lc[q].smalls[k] = 0;
        c->lc[q].tile_next = 0;
        c->lc[q].tab = 0;
        c->lc[q].keys = 0;
        if (nseg) c->levels += 1;
    }
}

// ---------------------------------------------------------------------------
// Plan kernel, level L.
//  (1) For every segment of level L: the pivot is the median of a sample of
//      the segment (Section 2: median of three, or of a larger sample).  The
//      sample is stratified -- one key from each of k equal strata, at a
//      hashed position inside the stratum -- so sorted, reversed and
//      periodic inputs still yield central pivots.
//  (2) Writes the equal-key runs recorded by level L-1 into X (keys: the
//      pivot bits; pairs: the payloads parked in the side buffer).
//  Block 0 also clears the counters of slot (L+1)&1, which the partition
//  kernel of level L fills.

template <int DT, int NT>
struct PlanLds {
    typename KeyT<DT>::raw samp[NT / 64][kMaxSample + 1];
    typename KeyT<DT>::raw grp[NT / 64][8];  // group medians (medians of medians)
    typename KeyT<DT>::raw pick[NT / 64];
    typename KeyT<DT>::raw bcast;            // wave 0's pivot, for the whole workgroup
};

// Sample of one segment of m keys at recursion depth `depth` (the paper's
// pivot strategies, Section 4): k samples; g > 0 means the pivot is the
// median of the k/g medians of g consecutive samples; otherwise it is the
// sample of rank `rk` (the median, or the 1/skew quantile of a skewed-pivot
// run).  Past the depth limit every strategy takes the median of the
// largest sample (the guard that keeps the recursion depth logarithmic).
struct PivotPlan {
    int k, g, rk;
};
__device__ inline PivotPlan pivot_plan(const Args& a, int64_t m, uint32_t depth) {
    PivotPlan pp{0, 0, 0};
    const int mode = a.pivot_mode;
    const bool deep = depth >= static_cast<uint32_t>(a.depth_limit);
    int64_t kk;
    if (!deep && mode == 3) {
        kk = 3;
    } else if (!deep && (mode == 5 || mode == 23)) {
        kk = mode;
    } else if (!deep && (mode == 33 || mode == 35 || mode == 55 || (mode == 1 && m < 20000))) {
        // medians of three (five) medians of three (five); the median of
        // sqrt(m) takes the median of five medians of five below 20000 keys
        const int outer = mode == 55 || mode == 1 ? 5 : 3;
        pp.g = mode == 33 ? 3 : 5;
        kk = outer * pp.g;
    } else if (!deep && mode == 1) {
        kk = static_cast<int64_t>(sqrt(static_cast<double>(m)));
        if (kk > a.sample_max) kk = a.sample_max;
    } else {
        // default: about sqrt(m)/4 samples within [7, sample_max]
        kk = deep ? a.sample_max : static_cast<int64_t>(sqrt(static_cast<double>(m))) / 4;
        if (kk > a.sample_max) kk = a.sample_max;
        if (kk < 7) kk = 7;
    }
    if (kk > m) {
        kk = m;
        pp.g = 0;
    }
    int k = static_cast<int>(kk) | 1;
    if (k > m) k -= 2;
    if (pp.g) k = static_cast<int>(kk);  // a whole number of groups (odd: 9, 15, 25)
    pp.k = k;
    pp.rk = (!deep && pp.g == 0 && a.pivot_skew >= 2) ? k / a.pivot_skew : k / 2;
    return pp;
}

// Element of rank `target` among the 64*P order keys a wave holds, P per
// lane (lane l holds positions P*l .. P*l+P-1): a bitonic sorting network
// over the wave -- partners less than P apart inside a lane's registers,
// farther ones in other lanes (lane xor) -- then the element at position
// `target`.  P = 1, 2 or 4: the network is sized to the sample.
template <class O, int P>
__device__ __forceinline__ O wave_rank_select(O (&v)[P], int target, int lane) {
    static_assert(P == 1 || P == 2 || P == 4, "one, two or four keys per lane");
#pragma unroll
    for (int size = 2; size <= 64 * P; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride < P) {
#pragma unroll
                for (int r = 0; r < P; ++r) {
                    const int pr = r ^ stride;
                    if (pr > r) {
                        const bool up = ((P * lane + r) & size) == 0;
                        const O x = v[r], y = v[pr];
                        const O lo = x < y ? x : y, hi = x < y ? y : x;
                        v[r] = up ? lo : hi;
                        v[pr] = up ? hi : lo;
                    }
                }
            } else {
                const int d = stride / P;
#pragma unroll
                for (int r = 0; r < P; ++r) {
                    const int pos = P * lane + r;
                    const O other = shfl_xor_o(v[r], d);
                    const bool keep_small = ((pos & stride) == 0) == ((pos & size) == 0);
                    v[r] = keep_small ? (other < v[r] ? other : v[r]) : (other > v[r] ? other : v[r]);
                }
            }
        }
    }
    const int r = target % P;
    O mine = v[0];
#pragma unroll
    for (int i = 1; i < P; ++i) mine = r == i ? v[i] : mine;
    if constexpr (sizeof(O) == 8) return static_cast<O>(bcast64(static_cast<uint64_t>(mine), target / P));
    else return static_cast<O>(__shfl(static_cast<int>(mine), target / P, 64));
}

// The sample of wave-held keys: sample i (of k <= 64*P) at position P*lane +
// r, past the sample the largest order key; its element of rank `target`.
template <class K, int P, class Pos>
__device__ __forceinline__ auto sample_rank_select(const typename K::raw* src, int k, int target, int lane,
                                                  Pos sample_pos) {
    using O = decltype(K::ord(typename K::raw()));
    O v[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const int i = P * lane + r;
        v[r] = i < k ? K::ord(src[sample_pos(i)]) : static_cast<O>(~O(0));
    }
    return wave_rank_select<O, P>(v, target, lane);
}

// The pivot of segment [lo, hi) at recursion depth `depth`, picked by wave
// wv of the workgroup from its own sample (all NT threads call this together:
// it holds workgroup barriers; `valid` false: the wave has no segment).
template <int DT, int NT>
__device__ typename KeyT<DT>::raw segment_pivot(const Args& a, const typename KeyT<DT>::raw* src, int64_t lo,
                                                int64_t hi, uint32_t depth, bool valid, PlanLds<DT, NT>& lds) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    using O = decltype(K::ord(R()));
    R* ws = lds.samp[wv];
    const int64_t m = hi - lo;
    const PivotPlan pp = valid ? pivot_plan(a, m, depth) : PivotPlan{0, 0, 0};
    const int k = pp.k;
    // sample i sits in stratum i at a hashed offset (first, middle and
    // last key for the median of three)
    auto sample_pos = [&](int i) -> int64_t {
        if (k == 3 && pp.g == 0) return i == 0 ? lo : (i == 1 ? lo + m / 2 : hi - 1);
        const int64_t stride = m / k;
        const uint64_t h = mix64((static_cast<uint64_t>(lo) * 0x9e3779b97f4a7c15ull) ^
                                 (static_cast<uint64_t>(hi) << 17) ^ (static_cast<uint64_t>(i) << 40) ^ depth);
        return lo + i * stride + static_cast<int64_t>(h % static_cast<uint64_t>(stride));
    };
    if (pp.g == 0) {
        // one sample: sorted in registers across the wave (a network of 64,
        // 128 or 256 keys, the smallest that holds it; none for a wave
        // without a segment); the pick is the key of the target rank
        O pick = 0;
        if (valid) {
            if (k <= 64) pick = sample_rank_select<K, 1>(src, k, pp.rk, lane, sample_pos);
            else if (k <= 128) pick = sample_rank_select<K, 2>(src, k, pp.rk, lane, sample_pos);
            else pick = sample_rank_select<K, 4>(src, k, pp.rk, lane, sample_pos);
        }
        // the workgroup's barriers stay the same for every wave (a wave with
        // medians of medians may share the workgroup)
        __syncthreads();
        __syncthreads();
        __syncthreads();
        __syncthreads();
        return K::inv(pick);
    }
    for (int i = lane; i < k; i += 64) ws[i] = src[sample_pos(i)];
    __syncthreads();
    // medians of medians: lane t takes the median of group t
    if (pp.g > 0 && lane < k / pp.g) {
        const R* grp = ws + lane * pp.g;
        R med = grp[0];
        for (int i = 0; i < pp.g; ++i) {
            const auto om = K::ord(grp[i]);
            int rank = 0;
            for (int j = 0; j < pp.g; ++j) {
                const auto oj = K::ord(grp[j]);
                rank += (oj < om) | ((oj == om) & (j < i));
            }
            if (rank == pp.g / 2) med = grp[i];
        }
        lds.grp[wv][lane] = med;
    }
    __syncthreads();
    // the pick: the candidate of the target rank (ties broken by index)
    const R* cand = pp.g > 0 ? lds.grp[wv] : ws;
    const int kc = pp.g > 0 ? k / pp.g : k;
    const int target = pp.g > 0 ? kc / 2 : pp.rk;
    for (int i = lane; i < kc; i += 64) {
        const R mine = cand[i];
        const auto om = K::ord(mine);
        int rank = 0;
#pragma unroll 8
        for (int j = 0; j < kc; ++j) {
            const auto oj = K::ord(cand[j]);
            rank += (oj < om) | ((oj == om) & (j < i));
        }
        if (rank == target) lds.pick[wv] = mine;
    }
    __syncthreads();
    const R piv = lds.pick[wv];
    __syncthreads();  // lds is free for the next call
    return piv;
}

// The plan step as workgroup `bid` of `nblk` (all NT threads).  Each
// segment's pivot goes into its descriptor and into the descriptors of its
// tiles (and the tiles' look-back words are cleared).  On the first levels,
// whose few segments have many tiles each, several workgroups of a segment
// each pick its pivot with one wave -- the pick is deterministic -- and write
// a share of its tile descriptors, so that a segment of many tiles is not
// left to one wave; otherwise one wave per segment.
constexpr uint32_t kPlanParts = 64;   // most plan workgroups that share one segment's tile descriptors
constexpr uint32_t kPlanDescs = 512;  // tile descriptors per plan workgroup on the first levels

template <int DT, class V, int NT>
__device__ void plan_body(const Args& a, int level, uint32_t bid, uint32_t nblk, PlanLds<DT, NT>& lds) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    constexpr int NW = NT / 64;  // one wave per segment
    static_assert(kMaxSample < 4 * 64, "a lane holds at most four samples");

    Ctl* c = a.ctl;
    const int p = level & 1, q = p ^ 1;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const unsigned long long lcs = c->lc[p].segs;
    uint32_t nseg = static_cast<uint32_t>(lcs);
    reset_next_slot(c, q, nseg, bid);
    if (nseg > a.cap_seg) nseg = a.cap_seg;  // an overflow was latched
    const R* src = static_cast<const R*>(p ? a.y_keys : a.x_keys);
    // workgroups per segment: one per kPlanDescs tile descriptors of the
    // average segment, at most kPlanParts and nblk / nseg (the others only
    // run the fills)
    uint32_t parts = 0;
    if (nseg > 0) {
        parts = static_cast<uint32_t>(lcs >> 32) / nseg / kPlanDescs;
        parts = parts < kPlanParts ? parts : kPlanParts;
        parts = parts < nblk / nseg ? parts : nblk / nseg;
    }

    if (parts >= 2) {
        // in each workgroup of a segment, wave 0 picks the pivot
        const uint32_t si = bid % nseg, part = bid / nseg;
        if (part < parts) {
            SegDesc* sd = &a.segs[p][si];
            const int64_t lo = sd->lo, hi = sd->hi;
            const uint32_t t0 = sd->t0, nt = sd->nt;
            const R pick0 = segment_pivot<DT, NT>(a, src, lo, hi, sd->depth, wv == 0, lds);
            if (tid == 0) lds.bcast = pick0;
            __syncthreads();
            const R pick = lds.bcast;
            // an in-place segment whose pivot its parent fixed keeps it
            const R piv = (sd->pad & kSegForced) ? static_cast<R>(sd->pivot_raw) : pick;
            const uint64_t po = static_cast<uint64_t>(K::ord(piv));
            if (part == 0 && tid == 0) {
                sd->pivot = po;
                sd->pivot_raw = static_cast<uint64_t>(piv);
                sd->cursor = 0;
            }
            TileDesc d;
            d.lo = lo;
            d.hi = hi;
            d.pivot = po;
            d.t0 = t0;
            d.si = si;
            const uint32_t j0 = static_cast<uint32_t>(static_cast<uint64_t>(nt) * part / parts);
            const uint32_t j1 = static_cast<uint32_t>(static_cast<uint64_t>(nt) * (part + 1) / parts);
            for (uint32_t j = j0 + tid; j < j1; j += NT) {
                a.tile_desc[t0 + j] = d;
                a.status[t0 + j] = 0;
            }
        }
    } else {
        // block-uniform trip count (the barriers inside); wave wv takes segment base + wv
        for (uint32_t base = bid * NW; base < nseg; base += nblk * NW) {
            const uint32_t si = base + wv;
            const bool valid = si < nseg;
            SegDesc* sd = &a.segs[p][valid ? si : 0];
            int64_t lo = 0, hi = 0;
            uint32_t depth = 0, t0 = 0, nt = 0;
            if (valid) {
                lo = sd->lo;
                hi = sd->hi;
                depth = sd->depth;
                t0 = sd->t0;
                nt = sd->nt;
            }
            const R pick = segment_pivot<DT, NT>(a, src, lo, hi, depth, valid, lds);
            if (valid) {
                const R piv = (sd->pad & kSegForced) ? static_cast<R>(sd->pivot_raw) : pick;
                if (lane == 0) {
                    sd->pivot = static_cast<uint64_t>(K::ord(piv));
                    sd->pivot_raw = static_cast<uint64_t>(piv);
                    sd->cursor = 0;
                }
                TileDesc d;
                d.lo = lo;
                d.hi = hi;
                d.pivot = static_cast<uint64_t>(K::ord(piv));
                d.t0 = t0;
                d.si = si;
                for (uint32_t j = lane; j < nt; j += 64) {
                    a.tile_desc[t0 + j] = d;
                    a.status[t0 + j] = 0;
                }
            }
        }
    }

    run_fills<DT, V, NT>(a, p, bid, nblk);
}

template <int DT, class V, int NT>
__global__ __launch_bounds__(NT) void k_plan(Args a) {
    __shared__ PlanLds<DT, NT> s_lds;
    if (a.ctl->error) return;  // an earlier step latched an error: the rest of the call does nothing
    plan_body<DT, V, NT>(a, a.level, blockIdx.x, gridDim.x, s_lds);
}

// N consecutive elements of 4 or 8 bytes from a 4-byte aligned address, in
// 16-byte (or 8-byte) vector loads; global memory takes unaligned vector
// accesses.
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));
template <class T, int N>
__device__ __forceinline__ void load_run(const T* p, T* out) {
    constexpr int B = N * static_cast<int>(sizeof(T));
    static_assert(B % 8 == 0, "whole 8-byte words");
    uint32_t w[B / 4];
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int q = 0; q < B / 16; ++q) {
            const u32x4_a4 v = reinterpret_cast<const u32x4_a4*>(p)[q];
            w[4 * q] = v.x;
            w[4 * q + 1] = v.y;
            w[4 * q + 2] = v.z;
            w[4 * q + 3] = v.w;
        }
    } else {
        const u32x2_a4 v = *reinterpret_cast<const u32x2_a4*>(p);
        w[0] = v.x;
        w[1] = v.y;
    }
    __builtin_memcpy(out, w, B);
}

// ---------------------------------------------------------------------------
// Partition tile, shared by the level-mode and persistent kernels.
//
// One workgroup partitions one tile of T = NT*EPT keys of a segment [lo, hi)
// around the segment's pivot: keys < pivot go to the left run, keys > pivot
// to the right run, keys == pivot are counted (keys) or parked in the side
// buffer (payloads).  Tile j of a segment covers [lo + j*T, +T) clipped to
// the segment (seg_tiles), so only its last tile is partial.  `status`
// points at the status words of the segment's tiles (index j).

__device__ __forceinline__ uint64_t cycles() { return static_cast<uint64_t>(clock64()); }

constexpr unsigned long long kLookbackTicks = 1ull << 27;  // ~1.3 s of the 100 MHz wall clock

struct TileIO {
    unsigned int* error;
    const void* src;
    void* dst;
    const void* vsrc;
    void* vdst;
    void* side;
    unsigned long long* status;
    unsigned long long* cursor;  // non-null: claim ranges with this cursor instead of the look-back
    int64_t lo, hi;
    uint64_t pivot;
    uint32_t j;
    uint32_t delay;  // stress test: sleep this many short periods before publishing the look-back status
};

struct TileOut {
    int64_t Lx, Gx;     // keys < pivot / > pivot in the segment's earlier tiles
    uint32_t nlt, ngt;  // this tile's counts
    bool last;          // this tile is the segment's last
    bool ok;            // the claimed ranges are consistent
};

// LDS of one partition tile: the staged keys (and payloads) plus T spare
// slots for keys that stay behind, the per-(item, wave) counts, the tile
// totals and the claimed offsets.  Kernels that run other work between tiles
// share this space with it.
template <int DT, class V, int NT, int EPT>
struct TileLds {
    static constexpr bool HV = !std::is_same<V, NoVal>::value;
    static constexpr int T = NT * EPT;
    static constexpr int NE = EPT * (NT / 64);
    // per-(item, wave) counts: less | greater (| equal for pairs) packed in
    // FW-bit fields; prefix sums stay below 2^FW
    using Cnt = typename std::conditional<HV, uint64_t, uint32_t>::type;
    static constexpr int FW = HV ? 21 : 16;
    typename KeyT<DT>::raw k[T + 64];
    typename ValStore<V>::type v[HV ? T + 64 : 1];
    Cnt cnt[NE];
    Cnt tot;
    int64_t ex[2];
};

template <int DT, class V, int NT, int EPT>
__device__ __forceinline__ TileOut tile_partition(const TileIO& io, unsigned long long* s_prof,
                                                  TileLds<DT, V, NT, EPT>& lds) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    using O = decltype(K::ord(R()));
    using VS = typename ValStore<V>::type;
    using Cls = typename std::conditional<(EPT <= 16), uint32_t, uint64_t>::type;
    using LT = TileLds<DT, V, NT, EPT>;
    constexpr bool HV = LT::HV;
    constexpr int T = LT::T;
    constexpr int NW = NT / 64;
    constexpr int NE = LT::NE;
    constexpr int C = (NE + 63) / 64;
    static_assert(EPT <= 32, "class codes are packed in 64 bits");
    using Cnt = typename LT::Cnt;
    constexpr int FW = LT::FW;
    constexpr Cnt FM = (Cnt(1) << FW) - 1;
    static_assert(T < (1 << FW), "tile counts must fit their packed fields");

    auto& s_k = lds.k;
    auto& s_v = lds.v;
    auto& s_cnt = lds.cnt;
    auto& s_tot = lds.tot;
    auto& s_ex = lds.ex;

    const int tid = static_cast<int>(threadIdx.x), lane = tid & 63, wv = tid >> 6;
    const bool prof = s_prof != nullptr;
    const uint64_t t_begin = prof ? cycles() : 0;
    const R* src = static_cast<const R*>(io.src);
    R* dst = static_cast<R*>(io.dst);
    const VS* vsrc = static_cast<const VS*>(io.vsrc);
    VS* vdst = static_cast<VS*>(io.vdst);
    VS* side = static_cast<VS*>(io.side);
    const uint32_t j = io.j;
    const int64_t tbase = io.lo + static_cast<int64_t>(j) * T;
    const int sl = 0;
    const int el = io.hi < tbase + T ? static_cast<int>(io.hi - tbase) : T;
    const bool full = sl == 0 && el == T;
    const O piv = static_cast<O>(io.pivot);
    const R* tsrc = src + tbase;

    // scanning phase: coalesced loads.  A whole tile in 16-byte loads:
    // thread tid holds the VW consecutive keys of vector u*NT + tid (u <
    // EPT/VW) as items u*VW .. u*VW+VW-1 (the order of the items only decides
    // the order of the keys inside the runs, the same on every run); a
    // partial tile item i of thread tid is key i*NT + tid
    R key[EPT];
    VS val[EPT];
    if (full) {
        constexpr int VW = 16 / static_cast<int>(sizeof(R));
        static_assert(EPT % VW == 0, "whole vectors per thread");
#pragma unroll
        for (int u = 0; u < EPT / VW; ++u) {
            const int64_t at = static_cast<int64_t>(u * NT + tid) * VW;
            load_run<R, VW>(tsrc + at, key + u * VW);
            if constexpr (HV) load_run<VS, VW>(vsrc + tbase + at, val + u * VW);
        }
    } else {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int off = i * NT + tid;
            const bool ok = off >= sl && off < el;
            key[i] = ok ? tsrc[off] : R(0);
            if constexpr (HV) val[i] = ok ? vsrc[tbase + off] : VS(0);
        }
    }
    // class codes (2 bits per item: 0 none, 1 less, 2 greater, 3 equal) and
    // per-(item, wave) counts from wave ballots
    Cls cls = 0;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const bool ok = full || ((i * NT + tid) >= sl && (i * NT + tid) < el);
        const O o = K::ord(key[i]);
        const bool lt = ok & (o < piv);
        const bool gt = ok & (o > piv);
        const uint64_t mlt = __ballot(lt), mgt = __ballot(gt);
        Cnt packed = static_cast<Cnt>(__popcll(mlt)) | (static_cast<Cnt>(__popcll(mgt)) << FW);
        if constexpr (HV) {
            const bool eq = ok & !lt & !gt;
            packed |= static_cast<Cnt>(__popcll(__ballot(eq))) << (2 * FW);
        }
        if (lane == 0) s_cnt[i * NW + wv] = packed;
        const Cls code = static_cast<Cls>(static_cast<uint32_t>(ok) * 3u - 2u * static_cast<uint32_t>(lt) -
                                          static_cast<uint32_t>(gt));
        cls |= code << (2 * i);
        // keep one item's lane masks live at a time (they live in SGPRs)
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    const uint64_t t_loaded = prof ? cycles() : 0;

    // offsets: exclusive prefix over (item, wave) counts, by wave 0
    if (wv == 0) {
        Cnt loc[C];
        Cnt sum = 0;
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
            const int idx = lane * C + cc;
            loc[cc] = idx < NE ? s_cnt[idx] : Cnt(0);
            sum += loc[cc];
        }
        const Cnt inc = static_cast<Cnt>(wave_inclusive_sum(static_cast<uint64_t>(sum), lane));
        Cnt run = inc - sum;
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
            const int idx = lane * C + cc;
            if (idx < NE) s_cnt[idx] = run;
            run += loc[cc];
        }
        if (lane == 63) s_tot = inc;
    }
    __syncthreads();
    const Cnt tot = s_tot;
    const uint32_t nlt = static_cast<uint32_t>(tot & FM);
    const uint32_t ngt = static_cast<uint32_t>((tot >> FW) & FM);
    const uint32_t neq = HV ? static_cast<uint32_t>((static_cast<uint64_t>(tot) >> (2 * FW)) & FM) : 0u;

    // wave 0 claims the output ranges while the other waves already stage
    // their keys in LDS: either with the segment's two cursors (one atomic
    // add moves the left cursor by nlt and the right one by ngt, the paper's
    // cursors l and r advancing a block at a time) or by a decoupled
    // look-back over the status words of the segment's earlier tiles (runs
    // laid out in tile order, so the layout is the same on every run)
    if (wv == 0) {
        const uint64_t t_lb = prof ? cycles() : 0;
        uint64_t Lx = 0, Gx = 0;
        unsigned long long* st_me = io.status + j;
        if (io.cursor) {
            if (lane == 0) {
                const unsigned long long got =
                    atomicAdd(io.cursor, (static_cast<unsigned long long>(ngt) << 32) | nlt);
                Lx = got & 0xffffffffull;
                Gx = got >> 32;
            }
        } else if (j == 0) {
            if (lane == 0) st_status(st_me, st_pack(kStInc, nlt, ngt));
        } else {
            for (uint32_t d = 0; d < io.delay; ++d) __builtin_amdgcn_s_sleep(16);
            if (lane == 0) st_status(st_me, st_pack(kStAgg, nlt, ngt));
            int64_t pos = static_cast<int64_t>(j) - 1;
            const unsigned long long t_wait = wall_clock64();
            bool stalled = false;
            for (;;) {
                const int64_t qq = pos - lane;
                uint64_t st;
                for (;;) {
                    st = (qq >= 0 && !stalled) ? ld_status(io.status + qq) : st_pack(kStInc, 0, 0);
                    if (prof && lane == 0) s_prof[2] += 1;
                    if (__ballot((st >> 62) == 0) == 0ull) break;
                    if (wall_clock64() - t_wait > kLookbackTicks) {
                        // a predecessor never published: latch the error and stop waiting
                        stalled = true;
                        if (lane == 0) atomicOr(io.error, ERR_STALL);
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (prof && lane == 0) s_prof[1] += 1;
                const uint64_t incm = __ballot((st >> 62) == kStInc);
                const int lim = incm ? (__ffsll(static_cast<unsigned long long>(incm)) - 1) : 63;
                const uint64_t l = lane <= lim ? ((st >> 31) & kM31) : 0ull;
                const uint64_t g = lane <= lim ? (st & kM31) : 0ull;
                Lx += wave_sum(l);
                Gx += wave_sum(g);
                if (incm) break;
                pos -= 64;
            }
            if (lane == 0) st_status(st_me, st_pack(kStInc, Lx + nlt, Gx + ngt));
        }
        if (lane == 0) {
            s_ex[0] = static_cast<int64_t>(Lx);
            s_ex[1] = static_cast<int64_t>(Gx);
        }
        if (prof && lane == 0) s_prof[3] += cycles() - t_lb;
    }

    // rearrangement, part 1: every key to its rank in LDS
    // [less run | greater run | equal run (pairs only)]; keys that stay
    // behind go to a per-lane spare slot, so the store needs no branch
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const uint32_t cl = static_cast<uint32_t>((cls >> (2 * i)) & Cls(3));
        const uint64_t mlt = __ballot(cl == 1), mgt = __ballot(cl == 2);
        const Cnt base = s_cnt[i * NW + wv];
        const int dl = static_cast<int>((base & FM) + mbcnt(mlt));
        const int dg = static_cast<int>(nlt + ((base >> FW) & FM) + mbcnt(mgt));
        int d = cl == 1 ? dl : (cl == 2 ? dg : T + lane);
        if constexpr (HV) {
            const uint64_t meq = __ballot(cl == 3);
            const int de = static_cast<int>(nlt + ngt + ((static_cast<uint64_t>(base) >> (2 * FW)) & FM) + mbcnt(meq));
            d = cl == 3 ? de : d;
            s_v[d] = val[i];
        }
        s_k[d] = key[i];
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();

    // rearrangement, part 2: coalesced copy of the runs to the other buffer
    TileOut out;
    out.Lx = s_ex[0];
    out.Gx = s_ex[1];
    out.nlt = nlt;
    out.ngt = ngt;
    out.last = tbase + el == io.hi;
    out.ok = out.Lx + nlt + out.Gx + ngt <= io.hi - io.lo;
    if (out.ok) {
        R* dl = dst + (io.lo + out.Lx);
        R* dr = dst + (io.hi - out.Gx - ngt);
        // streaming stores: the next level reads these keys only after the
        // whole pass (about 2 % faster than cached stores on full levels)
        for (int t = tid; t < static_cast<int>(nlt); t += NT) __builtin_nontemporal_store(s_k[t], dl + t);
        for (int t = tid; t < static_cast<int>(ngt); t += NT) __builtin_nontemporal_store(s_k[nlt + t], dr + t);
        if constexpr (HV) {
            VS* vl = vdst + (io.lo + out.Lx);
            VS* vr = vdst + (io.hi - out.Gx - ngt);
            for (int t = tid; t < static_cast<int>(nlt); t += NT) vl[t] = s_v[t];
            for (int t = tid; t < static_cast<int>(ngt); t += NT) vr[t] = s_v[nlt + t];
            const int64_t Ex = (tbase + sl - io.lo) - out.Lx - out.Gx;
            VS* ve = side + (io.lo + Ex);
            for (int t = tid; t < static_cast<int>(neq); t += NT) ve[t] = s_v[nlt + ngt + t];
        }
    }
    if (prof && tid == 0) {
        s_prof[0] += 1;
        s_prof[5] += t_loaded - t_begin;
        s_prof[4] += cycles() - t_begin;
    }
    return out;
}

// ---------------------------------------------------------------------------
// One tile of level `level` (all threads of the workgroup): the tile's
// segment, buffers and claim form, then the partition.
template <int DT, class V, int NT, int EPT>
__device__ __forceinline__ void tile_body(const Args& a, int level, uint32_t tile, const TileDesc& td,
                                          TileLds<DT, V, NT, EPT>& lds, unsigned long long* s_prof,
                                          uint32_t delay = 0) {
    Ctl* c = a.ctl;
    const int p = level & 1;
    const int tid = threadIdx.x;
    TileIO io;
    io.error = &c->error;
    io.src = p ? a.y_keys : a.x_keys;
    io.dst = p ? a.x_keys : a.y_keys;
    io.vsrc = p ? a.y_vals : a.x_vals;
    io.vdst = p ? a.x_vals : a.y_vals;
    io.side = a.side;
    io.status = a.status + td.t0;
    SegDesc* seg = &a.segs[p][td.si];
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    // payloads keep the look-back: their equal-key runs are parked by tile order
    const bool use_cursor = !HV && a.claim != 0;
    io.cursor = use_cursor ? &seg->cursor : nullptr;
    io.lo = td.lo;
    io.hi = td.hi;
    io.pivot = td.pivot;
    io.j = tile - td.t0;
    io.delay = delay;
    const TileOut r = tile_partition<DT, V, NT, EPT>(io, s_prof, lds);
    if (!r.ok && tid == 0) atomicOr(&c->error, ERR_OVERFLOW);  // inconsistent claim: nothing was written
}

// Partition kernel, level mode: one tile per workgroup.  Tiles are claimed in
// order through the level's ticket counter, so every tile that a look-back
// waits for is held by a running workgroup.
template <int DT, class V, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_partition(Args a) {
    __shared__ TileLds<DT, V, NT, EPT> s_lds;
    __shared__ TileDesc s_desc;
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_prof[6];
    Ctl* c = a.ctl;
    const int p = a.level & 1;
    const int tid = threadIdx.x;
    uint32_t ntiles = static_cast<uint32_t>(c->lc[p].segs >> 32);
    if (ntiles > a.cap_tile) ntiles = a.cap_tile;  // an overflow was latched
    // a launch may cover more workgroups than the level has tiles (a grid
    // fixed in advance); the surplus leaves before taking a ticket
    if (blockIdx.x >= ntiles || c->error) return;  // (an error latched by an earlier step: nothing runs)
    if (a.prof && tid < 6) s_prof[tid] = 0;
    // the look-back needs tiles taken in order (a ticket); cursor claims
    // wait for no other tile, so the workgroup index serves
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    const bool ticket = HV || a.claim == 0 || a.shuffle;
    if (tid == 0) {
        uint32_t t = ticket ? atomicAdd(&c->lc[p].tile_next, 1u) : blockIdx.x;
        if (a.shuffle && t < ntiles) {
            // stress test: tiles of each window of 64 tickets in reverse
            // order, so look-backs wait on tiles claimed after them (each
            // waits only inside its window, which the GPU holds at once)
            const uint32_t base = t & ~63u;
            const uint32_t w = ntiles - base < 64u ? ntiles - base : 64u;
            t = base + (w - 1u - (t - base));
        }
        s_tile = t;
        if (t < ntiles) s_desc = a.tile_desc[t];
    }
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) return;
    const TileDesc td = s_desc;
    // stress test: a pseudo-random pause before the look-back status is published
    const uint32_t delay = a.shuffle ? static_cast<uint32_t>(mix64(tile * 0x9e3779b97f4a7c15ull + a.level) & 31u) : 0u;
    tile_body<DT, V, NT, EPT>(a, a.level, tile, td, s_lds, a.prof ? s_prof : nullptr, delay);
    if (a.prof) {
        __syncthreads();
        if (tid < 6) atomicAdd(&c->prof[tid], s_prof[tid]);
    }
}

// Segment completion, level L (Section 2: the pivot leaves the recursion, the
// two sides recurse).  One thread per segment reads the segment's totals --
// the final cursor pair (cursor claims) or the inclusive status word of its
// last tile (look-back) -- and appends the equal run and the two children to
// the level L+1 lists.  Runs as its own launch after the partition launch, so
// every tile's claim and output is visible.  Appends are aggregated per wave:
// a wave prefix sum of the lanes' requests, one atomic add per wave and list.


// All 64 lanes: lane's first slot of a wave-wide append of `inc` to *ctr.
__device__ __forceinline__ uint64_t wave_append(unsigned long long* ctr, uint64_t inc, int lane) {
    const uint64_t incl = wave_inclusive_sum(inc, lane);
    const uint64_t total = bcast64(incl, 63);
    uint64_t base = 0;
    if (lane == 63 && total) base = atomicAdd(ctr, static_cast<unsigned long long>(total));
    return bcast64(base, 63) + incl - inc;
}

// The completion step as workgroup `bid` of `nblk` workgroups of 256 threads.
template <class V>
__device__ void complete_body(const Args& a, int level, uint32_t bid, uint32_t nblk) {
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    constexpr uint32_t WG = 256;
    Ctl* c = a.ctl;
    const int p = level & 1, q = p ^ 1;
    const int lane = lane_id();
    const bool cursor = !HV && a.claim != 0;
    uint32_t nseg = static_cast<uint32_t>(c->lc[p].segs);
    if (nseg > a.cap_seg) nseg = a.cap_seg;  // an overflow was latched
    const int64_t T = a.next_tile_keys;
    const int64_t S = a.small_cut;
    // statistics of this thread's appends: equal keys, and keys / tiles the
    // next level partitions
    unsigned long long fill_keys = 0, next_keys = 0, next_tiles = 0;
    // wave-uniform trip count: lanes past the list take part with nothing
    for (uint32_t base = bid * WG; base < nseg; base += nblk * WG) {
        const uint32_t si = base + threadIdx.x;
        const bool valid = si < nseg;
        int64_t lo = 0, hi = 0, Lt = 0, Gt = 0;
        uint32_t depth = 0, origin = 0;
        uint64_t raw = 0;
        if (valid) {
            const SegDesc sd = a.segs[p][si];
            lo = sd.lo;
            hi = sd.hi;
            depth = sd.depth + 1;
            raw = sd.pivot_raw;
            origin = sd.origin;
            if (cursor) {
                Lt = static_cast<int64_t>(sd.cursor & 0xffffffffull);
                Gt = static_cast<int64_t>(sd.cursor >> 32);
            } else {
                const uint64_t st = ld_status(&a.status[sd.t0 + sd.nt - 1]);
                Lt = static_cast<int64_t>((st >> 31) & kM31);
                Gt = static_cast<int64_t>(st & kM31);
            }
            if (Lt + Gt > hi - lo) {
                atomicOr(&c->error, ERR_OVERFLOW);
                Lt = Gt = 0;
                hi = lo;  // nothing to append
            }
        }
        const int64_t Et = (hi - lo) - Lt - Gt;
        // children: [lo, lo+Lt) and [hi-Gt, hi).  kind 1: partitioned at
        // L+1; kind 2: small sort; 0: nothing (empty, or one key already in
        // the caller's buffer)
        const int64_t clo[2] = {lo, hi - Gt};
        const int64_t chi[2] = {lo + Lt, hi};
        int kind[2], cls[2];
        uint32_t nt[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t m = chi[h] - clo[h];
            kind[h] = m <= 0 ? 0 : (m > S ? 1 : ((m == 1 && q == 0) ? 0 : 2));
            nt[h] = kind[h] == 1 ? seg_tiles(clo[h], chi[h], T) : 0u;
            cls[h] = kind[h] == 2 ? small_class(m) : -1;
            if (m == 1 && kind[h] == 0) mark_done(a, origin);  // one key, already in X
        }
        // segments of level L+1 (count | tiles << 32)
        const uint64_t sinc = static_cast<uint64_t>((kind[0] == 1) + (kind[1] == 1)) |
                              (static_cast<uint64_t>(nt[0] + nt[1]) << 32);
        if (__ballot(sinc != 0)) {
            const uint64_t at = wave_append(&c->lc[q].segs, sinc, lane);
            uint32_t idx = static_cast<uint32_t>(at);
            uint64_t t0 = at >> 32;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (kind[h] != 1) continue;
                if (idx >= a.cap_seg || t0 + nt[h] > a.cap_tile) {
                    atomicOr(&c->error, ERR_OVERFLOW);
                } else {
                    SegDesc d{};
                    d.lo = clo[h];
                    d.hi = chi[h];
                    d.t0 = static_cast<uint32_t>(t0);
                    d.nt = nt[h];
                    d.depth = depth;
                    d.origin = origin;
                    a.segs[q][idx] = d;
                }
                ++idx;
                t0 += nt[h];
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (kind[h] == 1) {
                next_keys += static_cast<unsigned long long>(chi[h] - clo[h]);
                next_tiles += nt[h];
            }
        }
        // small segments, per size class
        for (int k = 0; k < kSmallClasses; ++k) {
            const bool h0 = cls[0] == k, h1 = cls[1] == k;
            const uint64_t b0 = __ballot(h0), b1 = __ballot(h1);
            if ((b0 | b1) == 0) continue;
            const uint32_t total = static_cast<uint32_t>(__popcll(b0) + __popcll(b1));
            uint32_t first = 0;
            if (lane == 0) first = atomicAdd(&c->lc[q].smalls[k], total);
            first = static_cast<uint32_t>(__shfl(static_cast<int>(first), 0, 64));
            uint32_t idx = first + mbcnt(b0) + mbcnt(b1);
            SmallItem* dst = a.smalls[q] + static_cast<size_t>(k) * a.cap_small;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (cls[h] != k) continue;
                if (idx >= a.cap_small) atomicOr(&c->error, ERR_OVERFLOW);
                else dst[idx] = SmallItem{clo[h], chi[h], origin, 0u};
                ++idx;
            }
        }
        // equal run: written at level L+1 (keys: the pivot; pairs: the
        // payloads parked in the side buffer at [lo, lo + Et))
        const uint32_t nch = Et > 0 ? static_cast<uint32_t>((Et + kFillChunk - 1) / kFillChunk) : 0u;
        const uint64_t finc = Et > 0 ? (1ull | (static_cast<uint64_t>(nch) << 32)) : 0ull;
        if (__ballot(finc != 0)) {
            const uint64_t at = wave_append(&c->lc[q].fills, finc, lane);
            const uint32_t idx = static_cast<uint32_t>(at);
            if (Et > 0) {
                if (idx >= a.cap_fill) {
                    atomicOr(&c->error, ERR_OVERFLOW);
                } else {
                    FillItem f;
                    f.dst = lo + Lt;
                    f.len = Et;
                    f.side = lo;
                    f.raw = raw;
                    f.chunk0 = static_cast<uint32_t>(at >> 32);
                    f.origin = origin;
                    f.pad1 = 0;
                    a.fills[q][idx] = f;
                }
                fill_keys += static_cast<unsigned long long>(Et);
            }
        }
    }
    fill_keys = wave_sum(fill_keys);
    next_keys = wave_sum(next_keys);
    next_tiles = wave_sum(next_tiles);
    if (lane == 0) {
        if (fill_keys) atomicAdd(&c->fill_keys, fill_keys);
        if (next_keys) {
            atomicAdd(&c->part_keys, next_keys);
            atomicAdd(&c->lc[q].keys, next_keys);
            atomicAdd(&c->level_keys[level_slot(level + 1)], next_keys);
        }
        if (next_tiles) atomicAdd(&c->tiles, next_tiles);
    }
}

template <class V>
__global__ __launch_bounds__(256) void k_complete(Args a) {
    if (a.ctl->error) return;  // an earlier step latched an error: the rest of the call does nothing
    complete_body<V>(a, a.level, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Comparison sort of one small segment, the fallback of the bucket sort
// below for segments whose keys crowd into few buckets.
//
// A group of NTH threads sorts one segment of at most E*NTH keys: thread t
// holds items t*E .. t*E+E-1, sorts
// them with a bitonic network in registers (every merge of two sorted halves
// starts with the mirror step, item x against x ^ (2^k - 1), after which all
// compare-exchanges put the smaller item at the lower index), and the group
// merges the sorted runs through LDS (merge_sort below).  Padding items are
// larger than any key; pairs carry the key's index in the segment as a
// tie-break, which keeps padding behind real keys and makes the result
// unique.

template <class O, bool HV>
struct SItem;
template <class O>
struct SItem<O, false> {
    O k;
};
template <class O>
struct SItem<O, true> {
    O k;
    uint32_t i;
};

template <class O>
__device__ __forceinline__ bool item_less(const SItem<O, false>& a, const SItem<O, false>& b) {
    return a.k < b.k;
}
template <class O>
__device__ __forceinline__ bool item_less(const SItem<O, true>& a, const SItem<O, true>& b) {
    return (a.k < b.k) | ((a.k == b.k) & (a.i < b.i));
}

// a <- smaller, b <- larger.  Fields are selected one by one: a select
// between whole items would pick an address and keep the register arrays
// in private memory.
template <class O>
__device__ __forceinline__ void cx(SItem<O, false>& a, SItem<O, false>& b) {
    const O x = a.k, y = b.k;
    const bool s = y < x;
    a.k = s ? y : x;
    b.k = s ? x : y;
}
template <class O>
__device__ __forceinline__ void cx(SItem<O, true>& a, SItem<O, true>& b) {
    const O xk = a.k, yk = b.k;
    const uint32_t xi = a.i, yi = b.i;
    const bool s = (yk < xk) | ((yk == xk) & (yi < xi));
    a.k = s ? yk : xk;
    b.k = s ? xk : yk;
    a.i = s ? yi : xi;
    b.i = s ? xi : yi;
}

template <int E>
struct Log2 {
    static constexpr int value = 1 + Log2<E / 2>::value;
};
template <>
struct Log2<1> {
    static constexpr int value = 0;
};

// LDS slot of item x: one pad word per 32 (4-byte keys) or 16 (8-byte keys)
// items keeps the blocked-layout accesses free of bank conflicts.
template <class O>
__device__ __forceinline__ int lds_slot(int x) {
    return sizeof(O) == 4 ? x + (x >> 5) : x + (x >> 4);
}

// In-thread stages: register bit j (xor) and the mirror step of merge k.
template <class It, int E>
__device__ __forceinline__ void reg_xor(It (&v)[E], int j) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int pr = r ^ (1 << j);
        if (pr > r && pr < E) cx(v[r], v[pr]);
    }
}
template <class It, int E>
__device__ __forceinline__ void reg_mirror(It (&v)[E], int k) {
    const int m = (1 << k) - 1;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int pr = r ^ m;
        if (pr > r && pr < E) cx(v[r], v[pr]);
    }
}

// Merge sort of the P = E*NTH items of one group (the paper's Insertionsort
// stage replaced by a sort that suits a workgroup).  Each thread first sorts
// its E items in registers with a fully unrolled bitonic network, then the
// group merges runs pairwise through LDS, doubling the run length log2(NTH)
// times.  For a merge, a thread owns E consecutive outputs of the merged run:
// a merge-path binary search finds where they start in the two runs, then
// the thread produces them one by one, reading each next candidate from LDS.
// Items compare by key, and by index for pairs, so the order is total and
// the result unique.
template <class It, class O, int E>
__device__ __forceinline__ void reg_sort(It (&v)[E]) {
    constexpr int LE = Log2<E>::value;
#pragma unroll
    for (int k = 1; k <= LE; ++k) {
        reg_mirror(v, k);
#pragma unroll
        for (int j = k - 2; j >= 0; --j) reg_xor(v, j);
    }
}

template <class It, class O>
__device__ __forceinline__ It lds_item(const O* sk, const uint32_t* si, int x) {
    It it;
    it.k = sk[lds_slot<O>(x)];
    if constexpr (sizeof(It) > sizeof(O)) it.i = si[lds_slot<O>(x)];
    return it;
}

template <class O>
__device__ __forceinline__ void pick(SItem<O, false>& d, const SItem<O, false>& x, const SItem<O, false>& y,
                                     bool take_y) {
    d.k = take_y ? y.k : x.k;
}
template <class O>
__device__ __forceinline__ void pick(SItem<O, true>& d, const SItem<O, true>& x, const SItem<O, true>& y,
                                     bool take_y) {
    d.k = take_y ? y.k : x.k;
    d.i = take_y ? y.i : x.i;
}

template <class It, class O, int E, int NTH>
__device__ void merge_sort(It (&v)[E], int t, O* sk, uint32_t* si, int m) {
    // A thread owns outputs [t*E, t*E + E) at every level.  Positions at or
    // past m (the segment's size) hold padding at every level (padding sorts
    // after every real item), so a thread whose outputs all lie there has
    // nothing to do: its items and its LDS slots stay padding.  Whole waves
    // of a short segment in a large class then skip the merges.
    const bool idle = t * E >= m;
    if (!idle) reg_sort<It, O, E>(v);
#pragma unroll 1
    for (int L = E; L < E * NTH; L <<= 1) {
        __syncthreads();  // the previous level's reads are done
        if (!idle) {
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int x = t * E + r;
                sk[lds_slot<O>(x)] = v[r].k;
                if constexpr (sizeof(It) > sizeof(O)) si[lds_slot<O>(x)] = v[r].i;
            }
        }
        __syncthreads();
        if (idle) continue;
        // runs A = [base, base+L) and B = [base+L, base+2L); this thread's
        // outputs are positions [d, d+E) of the merged run
        const int per = (2 * L) / E;  // threads per merged run
        const int base = (t / per) * 2 * L;
        const int d = (t % per) * E;
        int lo = d > L ? d - L : 0, hi = d < L ? d : L;
        while (lo < hi) {  // merge path: how many of the first d outputs come from A
            const int mid = (lo + hi) >> 1;
            const It am = lds_item<It, O>(sk, si, base + mid);
            const It bm = lds_item<It, O>(sk, si, base + L + d - 1 - mid);
            if (item_less(bm, am)) hi = mid;
            else lo = mid + 1;
        }
        int a = lo, b = d - lo;
        It ka = lds_item<It, O>(sk, si, base + (a < L ? a : L - 1));
        It kb = lds_item<It, O>(sk, si, base + L + (b < L ? b : L - 1));
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const bool take_b = (b < L) & ((a >= L) | item_less(kb, ka));
            pick(v[r], ka, kb, take_b);
            a += take_b ? 0 : 1;
            b += take_b ? 1 : 0;
            // refill the consumed side (clamped inside the pair; an exhausted
            // side is never chosen again)
            const int nx = take_b ? (L + (b < L ? b : L - 1)) : (a < L ? a : L - 1);
            const It nxt = lds_item<It, O>(sk, si, base + nx);
            pick(kb, kb, nxt, take_b);
            pick(ka, ka, nxt, !take_b);
        }
    }
}

// LDS of the comparison sort (merge_sort) of one segment of at most E*NT
// keys, the fallback of the bucket sort below: keys (padded layout), the
// keys' indexes in the segment (pairs) and the staged payloads (pairs).
template <int DT, class V, int E, int NT>
struct SmallLds {
    using O = decltype(KeyT<DT>::ord(typename KeyT<DT>::raw()));
    static constexpr bool HV = !std::is_same<V, NoVal>::value;
    static constexpr int P = E * NT;       // items
    static constexpr int PS = P + P / 16;  // padded LDS items (covers both pad rules)
    O k[PS];
    uint32_t i[HV ? PS : 1];
    typename ValStore<V>::type v[HV ? P : 1];
};

// The comparison sort of one segment of m keys read from src[0, m) (pairs
// have staged their payloads in lds.v by position).  Writes the sorted
// segment (and payloads) to dst[0, m), dv[0, m).  Not inlined: the bucket
// sort calls it only for crowded segments, and its registers then do not
// weigh on the bucket sort's.
template <int DT, class V, int E, int NT>
__device__ __attribute__((noinline)) void compare_sort_segment(const typename KeyT<DT>::raw* src, int m,
                                                              SmallLds<DT, V, E, NT>& lds,
                                                              typename KeyT<DT>::raw* dst,
                                                              typename ValStore<V>::type* dv) {
    using K = KeyT<DT>;
    using SL = SmallLds<DT, V, E, NT>;
    using O = typename SL::O;
    constexpr bool HV = SL::HV;
    using It = SItem<O, HV>;
    O* sk = lds.k;
    uint32_t* si = lds.i;
    const int t = threadIdx.x;
    // keys in striped order (item r of thread t at position r*NT + t),
    // padding larger than any key at positions >= m
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = r * NT + t;
        sk[lds_slot<O>(x)] = x < m ? K::ord(src[x]) : static_cast<O>(~O(0));
        if constexpr (HV) si[lds_slot<O>(x)] = static_cast<uint32_t>(x);
    }
    __syncthreads();
    It v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = t * E + r;
        v[r].k = sk[lds_slot<O>(x)];
        if constexpr (HV) v[r].i = si[lds_slot<O>(x)];
    }
    merge_sort<It, O, E, NT>(v, t, sk, si, m);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = t * E + r;
        sk[lds_slot<O>(x)] = v[r].k;
        if constexpr (HV) si[lds_slot<O>(x)] = v[r].i;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = r * NT + t;
        if (x < m) {
            dst[x] = K::inv(sk[lds_slot<O>(x)]);
            if constexpr (HV) dv[x] = lds.v[si[lds_slot<O>(x)]];
        }
    }
}

// ---------------------------------------------------------------------------
// Small-segment sort (the paper's Insertionsort stage, Section 2, and its
// outlook on a better recursion stopper, Section 5).
//
// A segment that reaches the small sort is the key range between two
// pivots, so its keys are confined to [mn, mx].  One workgroup of NT
// threads sorts one segment of m <= E*NT keys in LDS:
//   1. keys are loaded (coalesced, striped, every load issued before any is
//      used) into registers; mn and mx are reduced across the workgroup;
//   2. every key goes to one of NB = 2^ceil(log2 m) buckets by a monotone
//      map of its order key: (x - mn) itself when the range is that small
//      (each bucket then holds one key value), else the high part of
//      (x - mn) * M with M about NB * 2^w / (range + 1), so that the keys
//      spread over the buckets in proportion to their values (about one
//      key per bucket for evenly spread keys);
//   3. bucket sizes are counted with LDS atomics (two 16-bit counters per
//      word), turned into bucket starts by a workgroup scan, and every key is
//      scattered to its bucket by an atomic increment of the bucket's cursor;
//      the keys are now ordered by bucket;
//   4. unless every bucket holds a single key value (keys only), the keys
//      inside each bucket are put in order by odd-even transposition rounds
//      over the whole segment -- each thread holds E consecutive keys in
//      registers and exchanges its edge keys with its neighbour lanes; keys
//      of different buckets are already in order and never swap, so c rounds
//      order every bucket of at most c keys -- and a short window around
//      each wave boundary is ordered by rank.  Pairs order equal keys by
//      their index in the segment, which makes the payload order
//      deterministic (equal keys keep their input order).
// A segment with a bucket of more than kBucketCap keys (skewed or heavily
// duplicated keys) is sorted by the comparison sort instead (merge_sort).
// The keys are exactly the segment's keys in ascending order either way.

constexpr int kBucketCap = 8;

template <int DT, class V, int NT, int SMAX>
struct BucketLds {
    static constexpr int E = SMAX / NT;
    using SL = SmallLds<DT, V, E, NT>;
    using O = typename SL::O;
    SL s;                                 // bucket arrays (s.k keys, s.i indexes) or the fallback's LDS
    uint32_t hist[SMAX / 2 + SMAX / 16];  // bucket counters, then cursors: 16 bits each, two per word (padded)
    O red[2][NT / 64];                    // per-wave min and max
    uint32_t wsum[NT / 64];               // per-wave scan totals
    uint32_t wmax[NT / 64];               // per-wave largest bucket
};

template <class O>
__device__ __forceinline__ O wave_min(O v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const O o = shfl_xor_o(v, d);
        v = o < v ? o : v;
    }
    return v;
}
template <class O>
__device__ __forceinline__ O wave_max(O v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const O o = shfl_xor_o(v, d);
        v = o > v ? o : v;
    }
    return v;
}

// LDS word of bucket counter pair w: one pad word per eight keeps the
// scan's per-thread runs of consecutive words on distinct banks.
__device__ __forceinline__ uint32_t hist_word(uint32_t w) { return w + (w >> 3); }

__device__ __forceinline__ uint32_t half16(const uint32_t* h, uint32_t b) {
    return (h[hist_word(b >> 1)] >> ((b & 1u) << 4)) & 0xffffu;
}

// LDS slot of position x of the bucket arrays: one pad item per sixteen.
__device__ __forceinline__ int bslot(int x) { return x + (x >> 4); }

__device__ __forceinline__ uint32_t mul_hi(uint32_t a, uint32_t b) { return __umulhi(a, b); }
__device__ __forceinline__ uint64_t mul_hi(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// One odd-even transposition round over items held E per thread in
// consecutive order (lane t holds positions E*t .. E*t+E-1 of its wave's
// run): even rounds pair (2i, 2i+1) inside each thread; odd rounds pair
// (2i+1, 2i+2) and the last item with the next lane's first.
template <class It, int E>
__device__ __forceinline__ void oet_round(It (&v)[E], bool odd, int lane) {
    if (!odd) {
#pragma unroll
        for (int i = 0; i + 1 < E; i += 2) cx(v[i], v[i + 1]);
    } else {
#pragma unroll
        for (int i = 1; i + 1 < E; i += 2) cx(v[i], v[i + 1]);
        It up, dn;
        if constexpr (sizeof(v[0].k) == 8) {
            dn.k = static_cast<decltype(v[0].k)>(shfl_down64(static_cast<uint64_t>(v[0].k), 1));
            up.k = static_cast<decltype(v[0].k)>(shfl_up64(static_cast<uint64_t>(v[E - 1].k), 1));
        } else {
            dn.k = static_cast<decltype(v[0].k)>(__shfl_down(static_cast<int>(v[0].k), 1, 64));
            up.k = static_cast<decltype(v[0].k)>(__shfl_up(static_cast<int>(v[E - 1].k), 1, 64));
        }
        if constexpr (sizeof(It) > sizeof(v[0].k)) {
            dn.i = static_cast<uint32_t>(__shfl_down(static_cast<int>(v[0].i), 1, 64));
            up.i = static_cast<uint32_t>(__shfl_up(static_cast<int>(v[E - 1].i), 1, 64));
        }
        if (lane < 63 && item_less(dn, v[E - 1])) v[E - 1] = dn;
        if (lane > 0 && item_less(v[0], up)) v[0] = up;
    }
}

// Sorts one segment [lo, lo + m) of buffer `src` (payloads `vsrc`) into the
// caller's arrays at lo (all NT threads of the workgroup).
// With `pr` (profile mode), thread 0 adds each phase's cycles to pr[0..4].
template <int DT, class V, int NT, int SMAX>
__device__ void bucket_sort_segment(const Args& a, int p, int64_t lo, int m, BucketLds<DT, V, NT, SMAX>& L,
                                    unsigned long long* pr) {
    uint64_t tp = pr ? cycles() : 0;
    auto mark = [&](int phase) {
        if (pr && threadIdx.x == 0) {
            const uint64_t t = cycles();
            pr[phase] += t - tp;
            tp = t;
        }
    };
    using K = KeyT<DT>;
    using R = typename K::raw;
    using BL = BucketLds<DT, V, NT, SMAX>;
    using O = typename BL::O;
    using VS = typename ValStore<V>::type;
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    using It = SItem<O, HV>;
    constexpr int E = BL::E;
    constexpr int NW = NT / 64;
    // opaque: keeps the per-item positions from being hoisted out of the
    // caller's loop over segments (and held in spilled registers across it)
    const int tid = opaque(static_cast<int>(threadIdx.x)), lane = tid & 63, wv = tid >> 6;
    const R* src = static_cast<const R*>(p ? a.y_keys : a.x_keys) + lo;
    const VS* vsrc = static_cast<const VS*>(p ? a.y_vals : a.x_vals) + lo;
    R* xk = static_cast<R*>(a.x_keys) + lo;
    VS* xv = static_cast<VS*>(a.x_vals) + lo;
    O* B = L.s.k;
    uint32_t* Bi = L.s.i;
    VS* sv = L.s.v;
    uint32_t* h = L.hist;

    // 1. load (positions past the segment read its last key and become
    // padding); the key range
    O key[E];
    {
        R raw[E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int x = r * NT + tid;
            raw[r] = src[x < m ? x : m - 1];
        }
        if constexpr (HV) {
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int x = r * NT + tid;
                if (x < m) sv[x] = vsrc[x];
            }
        }
#pragma unroll
        for (int r = 0; r < E; ++r) key[r] = K::ord(raw[r]);
    }
    O mn = key[0], mx = key[0];  // the clamped reads repeat keys of the segment
#pragma unroll
    for (int r = 1; r < E; ++r) {
        mn = key[r] < mn ? key[r] : mn;
        mx = key[r] > mx ? key[r] : mx;
    }
#pragma unroll
    for (int r = 0; r < E; ++r)
        if (r * NT + tid >= m) key[r] = static_cast<O>(~O(0));
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane == 0) {
        L.red[0][wv] = mn;
        L.red[1][wv] = mx;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        mn = L.red[0][w] < mn ? L.red[0][w] : mn;
        mx = L.red[1][w] > mx ? L.red[1][w] : mx;
    }
    mark(0);
    const O range = mx - mn;
    if (range == 0) {
        // one key value: the segment is sorted as it stands
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int x = r * NT + tid;
            if (x < m) {
                xk[x] = K::inv(key[r]);
                if constexpr (HV) xv[x] = sv[x];
            }
        }
        return;
    }
    // 2. the bucket map: NB = 2^hb >= m buckets
    const int hb = m > 1 ? 32 - __clz(m - 1) : 1;
    const uint32_t NB = 1u << hb;
    const bool exact = range < static_cast<O>(NB);
    O M = 0;
    if (!exact) {
        // about NB * 2^w / (range + 1); rounding only moves bucket borders
        // (the map stays monotone and is clamped below NB)
        const double q = static_cast<double>(NB) * (sizeof(O) == 8 ? 18446744073709551616.0 : 4294967296.0) /
                         (static_cast<double>(range) + 1.0);
        const double top = sizeof(O) == 8 ? 18446744073709551615.0 : 4294967295.0;
        M = q >= top ? static_cast<O>(~O(0)) : static_cast<O>(q);
    }
    auto bucket = [&](O x) -> uint32_t {
        const O d = x - mn;
        if (exact) return static_cast<uint32_t>(d);
        const O b = mul_hi(d, M);
        return b < static_cast<O>(NB - 1) ? static_cast<uint32_t>(b) : NB - 1;
    };
    const uint32_t nbw = (NB + 1u) >> 1;  // words of 16-bit counters
    for (uint32_t w = tid; w < nbw; w += NT) h[hist_word(w)] = 0u;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if (r * NT + tid < m) {
            const uint32_t b = bucket(key[r]);
            atomicAdd(&h[hist_word(b >> 1)], 1u << ((b & 1u) << 4));
        }
    }
    __syncthreads();
    mark(1);
    // 3. bucket starts: each thread scans a run of consecutive words (all
    // of its words read at once)
    constexpr int PW = SMAX / 2 / NT > 0 ? SMAX / 2 / NT : 1;  // most words per thread
    const uint32_t per = (nbw + NT - 1) / NT;
    const uint32_t w0 = tid * per;
    uint32_t cw[PW];
    uint32_t sum = 0, big = 0;
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const uint32_t w = w0 + i;
        cw[i] = (static_cast<uint32_t>(i) < per && w < nbw) ? h[hist_word(w)] : 0u;
    }
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const uint32_t c0 = cw[i] & 0xffffu, c1 = cw[i] >> 16;
        sum += c0 + c1;
        big = c0 > big ? c0 : big;
        big = c1 > big ? c1 : big;
    }
    const uint32_t inc = static_cast<uint32_t>(wave_inclusive_sum(static_cast<uint64_t>(sum), opaque(lane)));
    const uint32_t wbig = wave_max(big);
    if (lane == 63) L.wsum[wv] = inc;
    if (lane == 0) L.wmax[wv] = wbig;
    __syncthreads();
    uint32_t run = inc - sum;
    uint32_t maxc = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        run += w < wv ? L.wsum[w] : 0u;
        maxc = L.wmax[w] > maxc ? L.wmax[w] : maxc;
    }
    const bool order_step = !exact || HV;
    if (order_step && maxc > static_cast<uint32_t>(kBucketCap)) {
        // a crowded bucket: sort this segment by comparisons instead
        compare_sort_segment<DT, V, E, NT>(src, m, L.s, xk, xv);
        return;
    }
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const uint32_t w = w0 + i;
        const uint32_t s0 = run, s1 = run + (cw[i] & 0xffffu);
        run = s1 + (cw[i] >> 16);
        if (static_cast<uint32_t>(i) < per && w < nbw) h[hist_word(w)] = s0 | (s1 << 16);
    }
    __syncthreads();
    mark(2);
    // scatter into the buckets; each counter then holds its bucket's end
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = r * NT + tid;
        if (x < m) {
            const uint32_t b = bucket(key[r]);
            const uint32_t sh = (b & 1u) << 4;
            const uint32_t pos = (atomicAdd(&h[hist_word(b >> 1)], 1u << sh) >> sh) & 0xffffu;
            B[bslot(pos)] = key[r];
            if constexpr (HV) Bi[bslot(pos)] = static_cast<uint32_t>(x);
        }
    }
    __syncthreads();
    mark(3);
    if (!order_step) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int x = r * NT + tid;
            if (x < m) xk[x] = K::inv(B[bslot(x)]);
        }
        mark(4);
        return;
    }
    // 4. order inside the buckets by odd-even transposition: thread t holds
    // positions E*t .. E*t+E-1; keys of different buckets never swap, so
    // kBucketCap rounds order every bucket that lies inside one wave's run
    {
        It v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int x = E * tid + i;
            v[i].k = x < m ? B[bslot(x)] : static_cast<O>(~O(0));
            if constexpr (HV) v[i].i = x < m ? Bi[bslot(x)] : 0xffffffffu;
        }
        // a bucket of c keys is in order after c rounds
        const int rounds = static_cast<int>(maxc);
#pragma unroll
        for (int r = 0; r < kBucketCap; ++r)
            if (r < rounds) oet_round<It, E>(v, (r & 1) != 0, lane);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int x = E * tid + i;
            if (x < m) {
                B[bslot(x)] = v[i].k;
                if constexpr (HV) Bi[bslot(x)] = v[i].i;
            }
        }
    }
    __syncthreads();
    {
        // a bucket across a wave boundary lies within kBucketCap positions
        // of it: each position of that window is ranked inside the window
        constexpr int WIN = 2 * kBucketCap;
        const int wb = tid / WIN, wi = tid % WIN;
        const int b0 = (wb + 1) * 64 * E - kBucketCap;
        const bool fix = wb < NW - 1 && b0 + wi < m;
        It mine{};
        int dst = 0;
        if (fix) {
            mine.k = B[bslot(b0 + wi)];
            if constexpr (HV) mine.i = Bi[bslot(b0 + wi)];
            int rank = 0;
#pragma unroll 4
            for (int j = 0; j < WIN; ++j) {
                if (b0 + j < m) {
                    It y;
                    y.k = B[bslot(b0 + j)];
                    if constexpr (HV) y.i = Bi[bslot(b0 + j)];
                    rank += static_cast<int>(item_less(y, mine) | (!item_less(mine, y) & (j < wi)));
                }
            }
            dst = b0 + rank;
        }
        __syncthreads();
        if (fix) {
            B[bslot(dst)] = mine.k;
            if constexpr (HV) Bi[bslot(dst)] = mine.i;
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = r * NT + tid;
        if (x < m) {
            xk[x] = K::inv(B[bslot(x)]);
            if constexpr (HV) xv[x] = sv[Bi[bslot(x)]];
        }
    }
    mark(4);
}

// The small sort of level `level` as workgroup `bid` of `nblk`: every
// segment recorded for the level's small lists of the size classes up to
// small_class(SMAX) (largest class first, so that the long sorts start
// early), one per workgroup; CLO: the smallest class taken.
template <int DT, class V, int NT, int SMAX, int CLO = 0>
__device__ void small_all_body(const Args& a, int level, uint32_t bid, uint32_t nblk,
                               BucketLds<DT, V, NT, SMAX>& L) {
    constexpr int CHI = SMAX <= 64 ? 0 : (SMAX <= 128 ? 1 : (SMAX <= 256 ? 2 : (SMAX <= 512 ? 3 : (SMAX <= 1024 ? 4 :
                        (SMAX <= 2048 ? 5 : (SMAX <= 4096 ? 6 : (SMAX <= 8192 ? 7 : 8)))))));
    static_assert(CHI < kSmallClasses && CLO <= CHI, "size classes of the small lists");
    Ctl* c = a.ctl;
    const int p = level & 1;
    uint32_t cnt[kSmallClasses];
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < kSmallClasses; ++k) {
        // a count past the capacity means an overflow was latched; only the
        // items that were written are read
        cnt[k] = (k < CLO || k > CHI) ? 0u : (c->lc[p].smalls[k] < a.cap_small ? c->lc[p].smalls[k] : a.cap_small);
        total += cnt[k];
    }
    unsigned long long my_keys = 0;
    // profile mode: per-phase cycles of this workgroup's segments
    __shared__ unsigned long long s_pr[5];
    unsigned long long* pr = a.prof ? s_pr : nullptr;
    if (pr && threadIdx.x < 5) s_pr[threadIdx.x] = 0;
    uint32_t nseg = 0;
    for (uint32_t it = bid; it < total; it += nblk) {
        uint32_t r = it;
        int cls = CHI;
        while (r >= cnt[cls]) {
            r -= cnt[cls];
            --cls;
        }
        const SmallItem s = a.smalls[p][static_cast<size_t>(cls) * a.cap_small + r];
        const int m = static_cast<int>(s.hi - s.lo);
        bucket_sort_segment<DT, V, NT, SMAX>(a, p, s.lo, m, L, pr);
        my_keys += static_cast<unsigned long long>(m);
        ++nseg;
        __syncthreads();  // LDS is reused by the next segment (and every store is issued)
        if (threadIdx.x == 0) mark_done(a, s.origin);
    }
    if (threadIdx.x == 0 && my_keys) atomicAdd(&c->small_keys, my_keys);
    if (pr && threadIdx.x == 0 && nseg) {
        atomicAdd(&c->sprof[0], static_cast<unsigned long long>(nseg));
        for (int i = 0; i < 5; ++i) atomicAdd(&c->sprof[1 + i], s_pr[i]);
    }
}

// One launch sorts every small segment of a level.  512-thread workgroups
// get 128 VGPRs (two per CU): capped at 80 for a third one, the keys held in
// registers spill (measured on 2^28 int32 keys: 1.23 ms against 1.53 ms).
template <int DT, class V, int NT, int SMAX, int CLO>
__global__ __launch_bounds__(NT, NT >= 512 ? 4 : 3) void k_small(Args a) {
    __shared__ BucketLds<DT, V, NT, SMAX> s_lds;
    if (a.ctl->error) return;  // an earlier step latched an error: the rest of the call does nothing
    small_all_body<DT, V, NT, SMAX, CLO>(a, a.level, blockIdx.x, gridDim.x, s_lds);
}

// ---------------------------------------------------------------------------
// Persistent mode: the recursion of every level in one cooperative launch.
// The resident workgroups drain the level's device lists step by step --
// (1) pivots and tile descriptors, plus the equal runs and small sorts
// recorded by the previous level, (2) partition tiles claimed in order with
// the level's ticket counter, (3) segment completion, which appends the next
// level's lists -- with a grid-wide barrier after each step.  The loop ends
// on the device, at the first level with no segment left to partition, so
// the host waits once per sort.  The steps run the same code as the
// level-mode kernels.

constexpr unsigned long long kSpinTicks = 1ull << 27;  // ~1.3 s of the 100 MHz wall clock

// Waits (one thread) until the barrier generation reaches `want`; 0 when
// the wait ran out or another workgroup latched ERR_STALL.
__device__ inline int wait_gen(Ctl* c, uint32_t want) {
    const unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
        if (__hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_STALL) return 0;
        if (wall_clock64() - t0 > kSpinTicks) {
            atomicOr(&c->error, ERR_STALL);
            return 0;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return 1;
}

// Grid barriers.  On MI355X each XCD has its own L2, so a workgroup's
// writes become visible to the other XCDs only once that L2 is written back
// (agent-scope release), and a reader must drop what its CU and L2 hold
// (agent-scope acquire).  Every wait is bounded by the wall clock: a barrier
// that waits too long latches ERR_STALL, every other waiting workgroup sees
// it and gives up too, and the launch ends; the functions then return false
// in every thread and the caller leaves the kernel.

// Plain barrier (used once, to count the workgroups of each XCD): thread 0
// of each workgroup releases, counts itself in, and the last one to arrive
// opens the next generation.
__device__ inline bool grid_sync(Ctl* c, uint32_t nblk, uint32_t& gen, int* s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t want = gen + 1u;
        int ok = 1;
        __threadfence();
        const uint32_t prev = atomicAdd(&c->bar_arrive, 1u);
        if (prev == nblk - 1u) {
            __hip_atomic_store(&c->bar_arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&c->bar_gen, want, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = wait_gen(c, want);
        }
        __threadfence();
        gen = want;
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Barrier with one L2 writeback per XCD.  Every thread waits for its own
// stores to reach the L2; thread 0 then counts the workgroup in on its XCD's
// counter.  The XCD's last workgroup writes the (shared) L2 back once for all
// of them and counts the XCD in; the last XCD opens the next generation.
// Acquire stays per workgroup.  `my_n`: resident workgroups on this
// workgroup's XCD; `nxcd`: XCDs with resident workgroups.
// The opener also records the error word as it stands once every workgroup
// has arrived (bar_err); every workgroup reads that record, which nobody
// rewrites before the next barrier, so all of them agree on whether an
// error ends the launch here (an error written during a step is seen by
// all at the step's closing barrier, never by some workgroups earlier).
__device__ inline bool grid_sync_xcd(Ctl* c, uint32_t xcd, uint32_t my_n, uint32_t nxcd, uint32_t& gen, int* s_ok) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t want = gen + 1u;
        const uint32_t prev = atomicAdd(&c->xcd_arrive[xcd][0], 1u);
        if (prev == my_n - 1u) {
            __hip_atomic_store(&c->xcd_arrive[xcd][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (atomicAdd(&c->bar_arrive, 1u) == nxcd - 1u) {
                __hip_atomic_store(&c->bar_arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned err = __hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&c->bar_err, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&c->bar_gen, want, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        const int ok = wait_gen(c, want);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gen = want;
        *s_ok = ok && __hip_atomic_load(&c->bar_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Gives the segments of level slot p the tiles of the tile size a.tile_keys
// (first tile and tile count; the level's tile total).  Run by a single
// workgroup of NT threads: the tail kernel, whose first level may have been
// listed by multiway levels with their own tile size.
template <int NT>
__device__ void retile_level(const Args& a, int p) {
    __shared__ uint32_t s_w[NT / 64];
    Ctl* c = a.ctl;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t nseg = static_cast<uint32_t>(c->lc[p].segs);
    if (nseg > a.cap_seg) nseg = a.cap_seg;
    const int64_t T = a.tile_keys;
    uint64_t base = 0;
    for (uint32_t b = 0; b < nseg; b += NT) {
        const uint32_t i = b + tid;
        const uint32_t nt = i < nseg ? seg_tiles(a.segs[p][i].lo, a.segs[p][i].hi, T) : 0u;
        const uint32_t inc = static_cast<uint32_t>(wave_inclusive_sum(static_cast<uint64_t>(nt), opaque(lane)));
        if (lane == 63) s_w[wv] = inc;
        __syncthreads();
        uint64_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            before += w < wv ? s_w[w] : 0u;
            total += s_w[w];
        }
        if (i < nseg) {
            a.segs[p][i].t0 = static_cast<uint32_t>(base + before + inc - nt);
            a.segs[p][i].nt = nt;
        }
        base += total;
        __syncthreads();
    }
    if (tid == 0) {
        if (base > a.cap_tile) atomicOr(&c->error, ERR_OVERFLOW);
        c->lc[p].segs = (static_cast<unsigned long long>(base < a.cap_tile ? base : a.cap_tile) << 32) | nseg;
    }
    __syncthreads();
}

// LDS of the persistent kernel: one region that each step views as its own
// layout (steps are separated by barriers).
template <int DT, class V, int NT, int EPT, int SP>
struct PersistLds {
    static constexpr size_t mx(size_t x, size_t y) { return x > y ? x : y; }
    static constexpr size_t bytes =
        mx(mx(sizeof(TileLds<DT, V, NT, EPT>), sizeof(PlanLds<DT, NT>)), sizeof(BucketLds<DT, V, NT, SP>));
};

// Three workgroups per CU (2^28 int32 keys: 12.2 ms, against 15.7 ms at four
// with their registers capped at 128 and 14.6 ms at two without spills).
template <int DT, class V, int NT, int EPT, int SP>
__global__ __launch_bounds__(NT, 3) void k_persist(Args a) {
    static_assert(NT == 256, "the plan, map and completion steps run 256 threads");
    using PL = PersistLds<DT, V, NT, EPT, SP>;
    __shared__ alignas(16) unsigned char s_raw[PL::bytes];
    __shared__ TileDesc s_desc;
    __shared__ uint32_t s_tile;
    __shared__ int s_ok;
    Ctl* c = a.ctl;
    // errors latched by earlier launches (no workgroup of this one writes
    // before the first barrier): the same for every workgroup
    if (c->error) return;
    const uint32_t bid = blockIdx.x, nblk = gridDim.x;
    const int tid = threadIdx.x;
    const int level_cap = 4 * a.depth_limit + 64;
    uint32_t gen = 0;
    // count the workgroups of each XCD (hardware register XCC_ID)
    __shared__ uint32_t s_xn[2];
    const uint32_t xcd = static_cast<uint32_t>(__builtin_amdgcn_s_getreg((3 << 11) | 20)) % kMaxXcd;
    if (tid == 0) atomicAdd(&c->xcd_n[xcd], 1u);
    if (!grid_sync(c, nblk, gen, &s_ok)) return;
    if (tid == 0) {
        uint32_t nx = 0;
        for (int x = 0; x < kMaxXcd; ++x)
            nx += __hip_atomic_load(&c->xcd_n[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
        s_xn[0] = __hip_atomic_load(&c->xcd_n[xcd], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_xn[1] = nx;
    }
    __syncthreads();
    const uint32_t my_n = s_xn[0], nxcd = s_xn[1];
    for (int L = a.level;; ++L) {
        const int p = L & 1;
        if (L == a.level && a.retile) {
            retile_level<NT>(a, p);
            if (!grid_sync_xcd(c, xcd, my_n, nxcd, gen, &s_ok)) return;
        }
        const unsigned long long sc = c->lc[p].segs;
        const uint32_t nseg = static_cast<uint32_t>(sc);
        uint32_t ntile = static_cast<uint32_t>(sc >> 32);
        if (ntile > a.cap_tile) ntile = a.cap_tile;  // an overflow was latched
        // (1) pivots and tile descriptors of level L; equal runs and small
        // segments of level L-1
        plan_body<DT, V, NT>(a, L, bid, nblk, *reinterpret_cast<PlanLds<DT, NT>*>(s_raw));
        __syncthreads();
        small_all_body<DT, V, NT, SP>(a, L, bid, nblk, *reinterpret_cast<BucketLds<DT, V, NT, SP>*>(s_raw));
        __syncthreads();
        if (!grid_sync_xcd(c, xcd, my_n, nxcd, gen, &s_ok)) return;
        if (nseg == 0) break;
        if (L >= level_cap) {
            if (bid == 0 && tid == 0) atomicOr(&c->error, ERR_OVERFLOW);
            break;
        }
        // (2) partition tiles, claimed in order
        auto& tl = *reinterpret_cast<TileLds<DT, V, NT, EPT>*>(s_raw);
        for (;;) {
            if (tid == 0) {
                const uint32_t t = atomicAdd(&c->lc[p].tile_next, 1u);
                s_tile = t;
                if (t < ntile) s_desc = a.tile_desc[t];
            }
            __syncthreads();
            const uint32_t tile = s_tile;
            if (tile >= ntile) break;
            const TileDesc td = s_desc;
            tile_body<DT, V, NT, EPT>(a, L, tile, td, tl, nullptr);
            __syncthreads();  // the tile's LDS, s_tile and s_desc are free again
        }
        if (!grid_sync_xcd(c, xcd, my_n, nxcd, gen, &s_ok)) return;
        // (3) completion: the lists of level L+1
        complete_body<V>(a, L, bid, nblk);
        if (!grid_sync_xcd(c, xcd, my_n, nxcd, gen, &s_ok)) return;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers for one (dtype, payload, tile shape).  SMAX is the
// largest small segment (a power of two between 64 and 16384).

}  // namespace bqs

#include "bqs_multiway.hpp"
#include "bqs_inplace.hpp"

namespace bqs {

// multiway launchers (keys only), or nullptr without instantiating them.
// The per-tile kernels run 512 threads (twice the waves of the two-way tile,
// to hide the latency of their LDS work) over tiles of the two-way size,
// except that 8192-key tiles become 7168 keys (14 per thread): the scatter's
// LDS then fits four workgroups per CU instead of three (2^28 int32 keys:
// 8.4 instead of 9.0 ms).
template <int DT, int NT0, int EPT0, bool ON>
struct MultiFns {
    static constexpr int NT = 512;
    static constexpr int EPT = NT0 * EPT0 == 8192 ? 14 : NT0 * EPT0 / NT;
    static_assert(NT * EPT <= NT0 * EPT0 && EPT >= 1, "tiles no larger than the two-way step's");
    static constexpr int tile() { return NT * EPT; }
    static void plan(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_plan_multi<DT, NoVal, 256>), dim3(grid), dim3(256), 0, s, a);
    }
    static void count(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_mcount<DT, NT, EPT>), dim3(grid), dim3(NT), 0, s, a);
    }
    static void scan(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_mscan<DT, 256>), dim3(grid), dim3(256), 0, s, a);
    }
    static void scatter(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_mscatter<DT, NT, EPT>), dim3(grid), dim3(NT), 0, s, a);
    }
    using Fn = void (*)(const Args&, int, hipStream_t);
    static constexpr Fn p() { return &plan; }
    static constexpr Fn c() { return &count; }
    static constexpr Fn sc() { return &scan; }
    static constexpr Fn sa() { return &scatter; }
};
template <int DT, int NT, int EPT>
struct MultiFns<DT, NT, EPT, false> {
    static constexpr int tile() { return 0; }
    using Fn = void (*)(const Args&, int, hipStream_t);
    static constexpr Fn p() { return nullptr; }
    static constexpr Fn c() { return nullptr; }
    static constexpr Fn sc() { return nullptr; }
    static constexpr Fn sa() { return nullptr; }
};

template <int DT, class V, int NT, int EPT, int SMAX>
struct Launch {
    static constexpr int kPlanThreads = 256;
    static void plan(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_plan<DT, V, kPlanThreads>), dim3(grid), dim3(kPlanThreads), 0, s, a);
    }
    static void tile(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_partition<DT, V, NT, EPT>), dim3(grid), dim3(NT), 0, s, a);
    }
    // half-size tiles for keys-only levels of many segments (tiles of 32 KB
    // of keys: 8192 4-byte or 4096 8-byte keys)
    static constexpr bool kHalf =
        std::is_same<V, NoVal>::value && NT * EPT * sizeof(typename KeyT<DT>::raw) == 32768 && EPT % 2 == 0;
    static constexpr int kHalfEpt = kHalf ? EPT / 2 : EPT;
    static void tile_half(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_partition<DT, V, NT, kHalfEpt>), dim3(grid), dim3(NT), 0, s, a);
    }
    // double-size tiles on twice the threads for keys-only levels of few,
    // large segments
    static constexpr int kDoubleNt = kHalf ? 2 * NT : NT;
    static void tile_double(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_partition<DT, V, kDoubleNt, EPT>), dim3(grid), dim3(kDoubleNt), 0, s, a);
    }
    static void complete(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_complete<V>), dim3(grid), dim3(256), 0, s, a);
    }
    // small sort: 16 keys per thread (8 for pairs of 2048 keys), at least
    // 256 threads.  Cutoffs past 8192 keys get a second launch for the
    // largest class, on 1024 threads (one workgroup per CU), so that the
    // smaller segments keep workgroups of 512 threads (two per CU).
    static constexpr int kSmallMain = SMAX > 8192 ? 8192 : SMAX;
    static constexpr int kSmallThreads = kSmallMain / 16 < 256 ? 256 : kSmallMain / 16;
    static void small(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_small<DT, V, kSmallThreads, kSmallMain, 0>), dim3(grid), dim3(kSmallThreads), 0, s,
                           a);
        if constexpr (SMAX > 8192) {
            static_assert(SMAX == 16384, "one class past 8192 keys");
            hipLaunchKernelGGL((k_small<DT, V, 1024, SMAX, 8>), dim3(grid), dim3(1024), 0, s, a);
        }
    }
    static void map(const Args& a, int grid, hipStream_t s) { launch_map(a, grid, s); }
    // persistent mode: small segments up to 4096 keys (the classes whose
    // groups fit a 256-thread workgroup)
    static constexpr int kPersistSmall = SMAX < 4096 ? SMAX : 4096;
    static hipError_t persist(const Args& a, int grid, hipStream_t s) {
        void* args[] = {const_cast<Args*>(&a)};
        return hipLaunchCooperativeKernel(k_persist<DT, V, NT, EPT, kPersistSmall>, dim3(grid), dim3(NT), args, 0,
                                          s);
    }
    // the tail: the persistent kernel's loop on one workgroup, small segments
    // up to the full cutoff
    static void tail(const Args& a, hipStream_t s) {
        hipLaunchKernelGGL((k_persist<DT, V, NT, EPT, SMAX>), dim3(1), dim3(NT), 0, s, a);
    }
    // in-place levels (tiles of kIpT keys) and their one-workgroup tail
    static void ip_count(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_ip_count<DT, kIpNT, kIpEPT>), dim3(grid), dim3(kIpNT), 0, s, a);
    }
    static void ip_scan(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_ip_scan<256>), dim3(grid), dim3(256), 0, s, a);
    }
    static void ip_exchange(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_ip_exchange<DT, V, kIpNT, kIpEPT>), dim3(grid), dim3(kIpNT), 0, s, a);
    }
    static void ip_complete(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL(k_ip_complete<V>, dim3(grid), dim3(256), 0, s, a);
    }
    static void ip_tail(const Args& a, hipStream_t s) {
        hipLaunchKernelGGL((k_ip_tail<DT, V, kIpNT, kIpEPT, SMAX>), dim3(1), dim3(kIpNT), 0, s, a);
    }
    static int persist_blocks_per_cu() {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<DT, V, NT, EPT, kPersistSmall>, NT, 0) !=
            hipSuccess)
            return 0;
        return nb;
    }
    static const Ops* ops() {
        static const Ops o{
            NT * EPT,
            SMAX,
            // default cutoff: the largest in-LDS size (measured best on 2^28
            // uniform int32 keys)
            SMAX,
            &plan,
            &map,
            &small,
            &tile,
            &complete,
            MultiFns<DT, NT, EPT, std::is_same<V, NoVal>::value>::p(),
            MultiFns<DT, NT, EPT, std::is_same<V, NoVal>::value>::c(),
            MultiFns<DT, NT, EPT, std::is_same<V, NoVal>::value>::sc(),
            MultiFns<DT, NT, EPT, std::is_same<V, NoVal>::value>::sa(),
            &persist,
            &tail,
            &persist_blocks_per_cu,
            kPersistSmall,
            MultiFns<DT, NT, EPT, std::is_same<V, NoVal>::value>::tile(),
            &ip_count,
            &ip_scan,
            &ip_exchange,
            &ip_complete,
            &ip_tail,
            kHalf ? NT * EPT / 2 : 0,
            kHalf ? &tile_half : nullptr,
            kHalf ? 2 * NT * EPT : 0,
            kHalf ? &tile_double : nullptr};
        return &o;
    }
};

}  // namespace bqs
