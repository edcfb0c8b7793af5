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

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int d) {
    const int lo = __shfl_xor(static_cast<int>(static_cast<uint32_t>(v)), d, 64);
    const int hi = __shfl_xor(static_cast<int>(static_cast<uint32_t>(v >> 32)), d, 64);
    return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ __forceinline__ uint64_t wave_inclusive_sum(uint64_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t t = shfl_up64(v, d);
        if (lane >= d) v += t;
    }
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
// Work-list appends (one thread).  A segment of more than small_cut keys is
// partitioned at the next level; a shorter one is finished by the small
// sort; one key already in the caller's buffer needs nothing.

__device__ inline void push_segment(const Args& a, int slot, int64_t lo, int64_t hi,
                                    uint32_t depth) {
    const int64_t m = hi - lo;
    if (m <= 0) return;
    Ctl* c = a.ctl;
    if (m > a.small_cut) {
        const int64_t T = a.tile_keys;
        const uint32_t nt = static_cast<uint32_t>((hi + T - 1) / T - lo / T);
        const unsigned long long r =
            atomicAdd(&c->lc[slot].segs, (static_cast<unsigned long long>(nt) << 32) | 1ull);
        const uint32_t idx = static_cast<uint32_t>(r);
        const uint64_t t0 = r >> 32;
        if (idx >= a.cap_seg || t0 + nt > a.cap_tile) {
            atomicOr(&c->error, ERR_OVERFLOW);
            return;
        }
        SegDesc d;
        d.lo = lo;
        d.hi = hi;
        d.pivot = 0;
        d.pivot_raw = 0;
        d.t0 = static_cast<uint32_t>(t0);
        d.nt = nt;
        d.depth = depth;
        d.pad = 0;
        a.segs[slot][idx] = d;
    } else {
        if (m == 1 && slot == 0) return;
        const uint32_t idx = atomicAdd(&c->lc[slot].smalls, 1u);
        if (idx >= a.cap_small) {
            atomicOr(&c->error, ERR_OVERFLOW);
            return;
        }
        a.smalls[slot][idx] = SmallItem{lo, hi};
    }
}

__device__ inline void push_fill(const Args& a, int slot, int64_t dst, int64_t len, int64_t side,
                                 uint64_t raw) {
    if (len <= 0) return;
    Ctl* c = a.ctl;
    const uint32_t nch = static_cast<uint32_t>((len + kFillChunk - 1) / kFillChunk);
    const unsigned long long r =
        atomicAdd(&c->lc[slot].fills, (static_cast<unsigned long long>(nch) << 32) | 1ull);
    const uint32_t idx = static_cast<uint32_t>(r);
    if (idx >= a.cap_fill) {
        atomicOr(&c->error, ERR_OVERFLOW);
        return;
    }
    FillItem f;
    f.dst = dst;
    f.len = len;
    f.side = side;
    f.raw = raw;
    f.chunk0 = static_cast<uint32_t>(r >> 32);
    f.pad0 = 0;
    f.pad1 = 0;
    a.fills[slot][idx] = f;
    atomicAdd(&c->fill_keys, static_cast<unsigned long long>(len));
}

// ---------------------------------------------------------------------------
// Plan kernel, level L.
//  (1) For every segment of level L: the pivot is the median of a sample of
//      the segment (Section 2: median of three, or of a larger sample).  The
//      sample is stratified -- one key from each of k equal strata, at a
//      hashed position inside the stratum -- so sorted, reversed and
//      periodic inputs still yield central pivots.  The kernel then maps the
//      segment's tiles and clears their status words.
//  (2) Writes the equal-key runs recorded by level L-1 into X (keys: the
//      pivot bits; pairs: the payloads parked in the side buffer).
//  Block 0 also clears the counters of slot (L+1)&1, which the partition
//  kernel of level L fills.

template <int DT, class V, int NT>
__global__ __launch_bounds__(NT) void k_plan(Args a) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    static_assert(NT >= kMaxSample + 1, "one thread per sample");
    __shared__ R s_samp[kMaxSample + 1];
    __shared__ R s_pick;

    Ctl* c = a.ctl;
    const int p = a.level & 1, q = p ^ 1;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) {
        c->lc[q].segs = 0;
        c->lc[q].fills = 0;
        c->lc[q].smalls = 0;
        c->lc[q].tile_next = 0;
    }
    const uint32_t nseg = static_cast<uint32_t>(c->lc[p].segs);
    const R* src = static_cast<const R*>(p ? a.y_keys : a.x_keys);

    for (uint32_t si = blockIdx.x; si < nseg; si += gridDim.x) {
        SegDesc* sd = &a.segs[p][si];
        const int64_t lo = sd->lo, hi = sd->hi, m = hi - lo;
        const uint32_t depth = sd->depth;
        int k;
        if (a.pivot_mode == 3 && depth < static_cast<uint32_t>(a.depth_limit)) {
            k = 3;
        } else {
            // about sqrt(m)/4 samples, odd, within [7, sample_max]; past the
            // depth limit the largest sample is used
            int64_t kk = static_cast<int64_t>(sqrt(static_cast<double>(m))) / 4;
            if (depth >= static_cast<uint32_t>(a.depth_limit)) kk = a.sample_max;
            if (kk > a.sample_max) kk = a.sample_max;
            if (kk < 7) kk = 7;
            if (kk > m) kk = m;
            k = static_cast<int>(kk) | 1;
            if (k > m) k -= 2;
        }
        if (tid < k) {
            int64_t pos;
            if (k == 3) {
                pos = tid == 0 ? lo : (tid == 1 ? lo + m / 2 : hi - 1);
            } else {
                const int64_t stride = m / k;
                const uint64_t h = mix64((static_cast<uint64_t>(lo) * 0x9e3779b97f4a7c15ull) ^
                                         (static_cast<uint64_t>(hi) << 17) ^
                                         (static_cast<uint64_t>(tid) << 40) ^ depth);
                pos = lo + tid * stride + static_cast<int64_t>(h % static_cast<uint64_t>(stride));
            }
            s_samp[tid] = src[pos];
        }
        __syncthreads();
        if (tid < k) {
            // rank of this sample: smaller samples, plus equal ones of lower index
            const R mine = s_samp[tid];
            const auto om = K::ord(mine);
            int rank = 0;
            for (int j = 0; j < k; ++j) {
                const auto oj = K::ord(s_samp[j]);
                rank += (oj < om) | ((oj == om) & (j < tid));
            }
            if (rank == k / 2) s_pick = mine;
        }
        __syncthreads();
        const R piv = s_pick;
        if (tid == 0) {
            sd->pivot = static_cast<uint64_t>(K::ord(piv));
            sd->pivot_raw = static_cast<uint64_t>(piv);
            atomicAdd(&c->part_keys, static_cast<unsigned long long>(m));
            atomicAdd(&c->tiles, static_cast<unsigned long long>(sd->nt));
        }
        const uint32_t t0 = sd->t0, nt = sd->nt;
        for (uint32_t t = tid; t < nt; t += NT) {
            a.tile_seg[t0 + t] = si;
            a.status[t0 + t] = 0;
        }
        __syncthreads();
    }

    // equal-key runs of the previous level
    const unsigned long long fc = c->lc[p].fills;
    const uint32_t nfill = static_cast<uint32_t>(fc);
    const uint32_t nchunk = static_cast<uint32_t>(fc >> 32);
    R* xk = static_cast<R*>(a.x_keys);
    for (uint32_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        // items are ordered by chunk0: find the last one starting at or before ch
        uint32_t lo_i = 0, hi_i = nfill;
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
    }
}

// ---------------------------------------------------------------------------
// Partition kernel, level L: one tile of T = NT*EPT keys per iteration.
// Tiles are claimed in order through an atomic counter, so every tile that
// a look-back waits for is held by a running workgroup.

template <int DT, class V, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_partition(Args a) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    using VS = typename ValStore<V>::type;
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    constexpr int T = NT * EPT;
    constexpr int NW = NT / 64;
    constexpr int NE = EPT * NW;
    constexpr int C = (NE + 63) / 64;
    static_assert(T < (1 << 21), "tile counts are packed in 21 bits");
    static_assert(EPT <= 32, "class codes are packed in 64 bits");

    __shared__ R s_k[T];
    __shared__ VS s_v[HV ? T : 1];
    __shared__ uint64_t s_cnt[NE];
    __shared__ uint64_t s_tot;
    __shared__ uint32_t s_tile;
    __shared__ int64_t s_ex[2];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    Ctl* c = a.ctl;
    const int p = a.level & 1, q = p ^ 1;
    const uint32_t ntiles = static_cast<uint32_t>(c->lc[p].segs >> 32);
    const R* src = static_cast<const R*>(p ? a.y_keys : a.x_keys);
    R* dst = static_cast<R*>(p ? a.x_keys : a.y_keys);
    const VS* vsrc = static_cast<const VS*>(p ? a.y_vals : a.x_vals);
    VS* vdst = static_cast<VS*>(p ? a.x_vals : a.y_vals);
    VS* side = static_cast<VS*>(a.side);
    const SegDesc* segs = a.segs[p];

    for (;;) {
        if (tid == 0) s_tile = atomicAdd(&c->lc[p].tile_next, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) return;
        const SegDesc sd = segs[a.tile_seg[tile]];
        const uint32_t j = tile - sd.t0;
        // tiles sit on multiples of T in the array, so full tiles are aligned
        const int64_t tbase = (sd.lo / T + j) * static_cast<int64_t>(T);
        const int64_t s = sd.lo > tbase ? sd.lo : tbase;
        const int64_t e = sd.hi < tbase + T ? sd.hi : tbase + T;
        const auto piv = static_cast<decltype(K::ord(R()))>(sd.pivot);

        // scanning phase: coalesced loads, item i of thread tid is key tbase + i*NT + tid
        R key[EPT];
        VS val[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int64_t pos = tbase + i * NT + tid;
            const bool ok = pos >= s && pos < e;
            key[i] = ok ? src[pos] : R(0);
            if constexpr (HV) val[i] = ok ? vsrc[pos] : VS(0);
        }
        uint64_t cls = 0;  // 2 bits per item: 0 none, 1 less, 2 greater, 3 equal
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int64_t pos = tbase + i * NT + tid;
            const bool ok = pos >= s && pos < e;
            const auto o = K::ord(key[i]);
            const bool lt = ok & (o < piv);
            const bool gt = ok & (o > piv);
            const bool eq = ok & !lt & !gt;
            const uint64_t mlt = __ballot(lt), mgt = __ballot(gt);
            const uint64_t meq = HV ? __ballot(eq) : 0ull;
            if (lane == 0)
                s_cnt[i * NW + wv] = static_cast<uint64_t>(__popcll(mlt)) |
                                     (static_cast<uint64_t>(__popcll(mgt)) << 21) |
                                     (static_cast<uint64_t>(__popcll(meq)) << 42);
            const uint64_t code = lt ? 1ull : (gt ? 2ull : (eq ? 3ull : 0ull));
            cls |= code << (2 * i);
        }
        __syncthreads();

        // offsets: exclusive prefix over (item, wave) counts, by wave 0
        if (wv == 0) {
            uint64_t loc[C];
            uint64_t sum = 0;
#pragma unroll
            for (int cc = 0; cc < C; ++cc) {
                const int idx = lane * C + cc;
                loc[cc] = idx < NE ? s_cnt[idx] : 0ull;
                sum += loc[cc];
            }
            const uint64_t inc = wave_inclusive_sum(sum);
            uint64_t run = inc - sum;
#pragma unroll
            for (int cc = 0; cc < C; ++cc) {
                const int idx = lane * C + cc;
                if (idx < NE) s_cnt[idx] = run;
                run += loc[cc];
            }
            if (lane == 63) s_tot = inc;
        }
        __syncthreads();
        const uint64_t tot = s_tot;
        const uint32_t nlt = static_cast<uint32_t>(tot & kM21);
        const uint32_t ngt = static_cast<uint32_t>((tot >> 21) & kM21);
        const uint32_t neq = static_cast<uint32_t>((tot >> 42) & kM21);

        // wave 0 claims the output ranges (look-back) while the other waves
        // already stage their keys in LDS
        if (wv == 0) {
            uint64_t Lx = 0, Gx = 0;
            if (j == 0) {
                if (lane == 0) st_status(&a.status[tile], st_pack(kStInc, nlt, ngt));
            } else {
                if (lane == 0) st_status(&a.status[tile], st_pack(kStAgg, nlt, ngt));
                int64_t pos = static_cast<int64_t>(tile) - 1;
                const int64_t first = sd.t0;
                for (;;) {
                    const int64_t qq = pos - lane;
                    uint64_t st;
                    for (;;) {
                        st = qq >= first ? ld_status(&a.status[qq]) : st_pack(kStInc, 0, 0);
                        if (__ballot((st >> 62) == 0) == 0ull) break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    const uint64_t incm = __ballot((st >> 62) == kStInc);
                    const int lim = incm ? (__ffsll(static_cast<unsigned long long>(incm)) - 1) : 63;
                    const uint64_t l = lane <= lim ? ((st >> 31) & kM31) : 0ull;
                    const uint64_t g = lane <= lim ? (st & kM31) : 0ull;
                    Lx += wave_sum(l);
                    Gx += wave_sum(g);
                    if (incm) break;
                    pos -= 64;
                }
                if (lane == 0) st_status(&a.status[tile], st_pack(kStInc, Lx + nlt, Gx + ngt));
            }
            if (lane == 0) {
                s_ex[0] = static_cast<int64_t>(Lx);
                s_ex[1] = static_cast<int64_t>(Gx);
            }
        }

        // rearrangement, part 1: every key to its rank in LDS
        // [less run | greater run | equal run (pairs only)]
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const uint32_t cl = static_cast<uint32_t>((cls >> (2 * i)) & 3ull);
            const uint64_t mlt = __ballot(cl == 1), mgt = __ballot(cl == 2);
            const uint64_t meq = HV ? __ballot(cl == 3) : 0ull;
            const uint64_t base = s_cnt[i * NW + wv];
            int d = -1;
            if (cl == 1) d = static_cast<int>((base & kM21) + mbcnt(mlt));
            else if (cl == 2) d = static_cast<int>(nlt + ((base >> 21) & kM21) + mbcnt(mgt));
            else if (HV && cl == 3) d = static_cast<int>(nlt + ngt + ((base >> 42) & kM21) + mbcnt(meq));
            if (d >= 0) {
                s_k[d] = key[i];
                if constexpr (HV) s_v[d] = val[i];
            }
        }
        __syncthreads();

        // rearrangement, part 2: coalesced copy of the runs to the other buffer
        const int64_t Lx = s_ex[0], Gx = s_ex[1];
        if (Lx + nlt + Gx + ngt > sd.hi - sd.lo) {
            // inconsistent look-back result: report it and write nothing
            if (tid == 0) atomicOr(&c->error, ERR_OVERFLOW);
            __syncthreads();
            continue;
        }
        const int64_t left0 = sd.lo + Lx;
        const int64_t right0 = sd.hi - Gx - ngt;
        const int nmove = static_cast<int>(nlt + ngt);
        for (int t = tid; t < nmove; t += NT) {
            const int64_t d = t < static_cast<int>(nlt) ? left0 + t : right0 + (t - static_cast<int>(nlt));
            dst[d] = s_k[t];
            if constexpr (HV) vdst[d] = s_v[t];
        }
        if constexpr (HV) {
            const int64_t Ex = (s - sd.lo) - Lx - Gx;
            for (int t = tid; t < static_cast<int>(neq); t += NT) side[sd.lo + Ex + t] = s_v[nmove + t];
        }

        // segment completion: the segment's last tile knows the totals
        if (j + 1 == sd.nt && tid == 0) {
            const int64_t Lt = Lx + nlt, Gt = Gx + ngt;
            const int64_t Et = (sd.hi - sd.lo) - Lt - Gt;
            push_fill(a, q, sd.lo + Lt, Et, sd.lo, sd.pivot_raw);
            push_segment(a, q, sd.lo, sd.lo + Lt, sd.depth + 1);
            push_segment(a, q, sd.hi - Gt, sd.hi, sd.depth + 1);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Small-segment sort (the paper's Insertionsort stage, Section 2): one
// workgroup loads a whole segment of at most SMAX keys into LDS as order
// keys, sorts it with a bitonic network, and writes it to X.  Pairs carry
// the key's index in the segment as a tie-break (so the network is stable
// and padding never displaces a real payload) and gather payloads from LDS.

template <int DT, class V, int NT, int SMAX>
__global__ __launch_bounds__(NT) void k_small(Args a) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    using VS = typename ValStore<V>::type;
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    __shared__ R s_o[SMAX];
    __shared__ uint32_t s_i[HV ? SMAX : 1];
    __shared__ VS s_v[HV ? SMAX : 1];

    Ctl* c = a.ctl;
    const int p = a.level & 1;
    const int tid = threadIdx.x;
    const uint32_t nsm = c->lc[p].smalls;
    const R* src = static_cast<const R*>(p ? a.y_keys : a.x_keys);
    R* xk = static_cast<R*>(a.x_keys);
    const VS* vsrc = static_cast<const VS*>(p ? a.y_vals : a.x_vals);
    VS* xv = static_cast<VS*>(a.x_vals);

    for (uint32_t it = blockIdx.x; it < nsm; it += gridDim.x) {
        const SmallItem si = a.smalls[p][it];
        const int m = static_cast<int>(si.hi - si.lo);
        int P = 1;
        while (P < m) P <<= 1;
        for (int t = tid; t < P; t += NT) {
            if (t < m) {
                s_o[t] = K::ord(src[si.lo + t]);
                if constexpr (HV) s_v[t] = vsrc[si.lo + t];
            } else {
                s_o[t] = static_cast<R>(~R(0));
            }
            if constexpr (HV) s_i[t] = static_cast<uint32_t>(t);
        }
        __syncthreads();
        for (int kk = 2; kk <= P; kk <<= 1) {
            for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int t = tid; t < (P >> 1); t += NT) {
                    const int i = 2 * t - (t & (jj - 1));
                    const int l = i + jj;
                    const bool up = (i & kk) == 0;
                    const R oa = s_o[i], ob = s_o[l];
                    bool gt;
                    if constexpr (HV) {
                        const uint32_t ia = s_i[i], ib = s_i[l];
                        gt = (oa > ob) | ((oa == ob) & (ia > ib));
                        if (gt == up) {
                            s_o[i] = ob;
                            s_o[l] = oa;
                            s_i[i] = ib;
                            s_i[l] = ia;
                        }
                    } else {
                        gt = oa > ob;
                        if (gt == up) {
                            s_o[i] = ob;
                            s_o[l] = oa;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int t = tid; t < m; t += NT) {
            xk[si.lo + t] = K::inv(s_o[t]);
            if constexpr (HV) xv[si.lo + t] = s_v[s_i[t]];
        }
        if (tid == 0) atomicAdd(&c->small_keys, static_cast<unsigned long long>(m));
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers for one (dtype, payload, tile shape).

template <int DT, class V, int NT, int EPT, int SMAX>
struct Launch {
    static constexpr int kPlanThreads = 256;
    static constexpr int kSmallThreads = 256;
    static void plan(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_plan<DT, V, kPlanThreads>), dim3(grid), dim3(kPlanThreads), 0, s, a);
    }
    static void small(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_small<DT, V, kSmallThreads, SMAX>), dim3(grid), dim3(kSmallThreads), 0,
                           s, a);
    }
    static void tile(const Args& a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_partition<DT, V, NT, EPT>), dim3(grid), dim3(NT), 0, s, a);
    }
    static const Ops* ops() {
        static const Ops o{NT * EPT, SMAX, &plan, &small, &tile};
        return &o;
    }
};

}  // namespace bqs
