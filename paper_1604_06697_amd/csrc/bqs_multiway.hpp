// Multiway partition step (keys only): one pass splits a segment around up to
// kSplit splitters instead of one pivot.  This is a sample-sort step,
// pointed to by the paper's related work on super scalar sample sort and its
// multi-pivot outlook (Sections 1 and 5); the default two-way step stays the
// paper's block partition.
//
// Buckets.  With u distinct splitters s_0 < ... < s_{u-1} (drawn from a
// sample of the segment), key x falls in bucket 2i + e, where i is the number
// of splitters below x and e = 1 when x equals s_i.  Odd buckets hold keys
// equal to a splitter: they are final and never recurse.  Every even bucket
// misses at least one key of the segment (a splitter), so each pass shrinks
// the problem -- the same argument as for the three-way split of the
// two-way step.
//
// One pass over a level, with the level's tiles laid out as in the two-way
// step (tile j of a segment covers [lo + j*T, +T) clipped to it):
//   k_mcount   per tile: bucket histogram (read 4 B / key); each (tile,
//              bucket) claims its offset inside the bucket with one atomic
//              add on the segment's bucket cursor (the paper's cursors, one
//              per bucket; tiles land in claim order, which leaves the
//              sorted keys unchanged);
//   k_mscan    per segment (one wave): bucket starts from the final cursors,
//              and the next level's lists (children, equal runs);
//   k_mscatter per tile: re-reads the keys, stages them in LDS by bucket and
//              writes every bucket's run coalesced to the other buffer.
#pragma once

namespace bqs {

constexpr int kSplit = 15;                 // splitters per segment, at most
constexpr int kBuckets = 2 * kSplit + 1;   // 31
constexpr int kBStride = 32;               // per-tile histogram / offset stride

// Bucket of order key o; s: 16 splitters (order keys) ascending, the unused
// tail set to the largest key; u: number in use.
__device__ __forceinline__ int bucket_of(uint64_t o, const uint64_t* s, int u) {
    int pos = 0;
#pragma unroll
    for (int step = 8; step >= 1; step >>= 1) pos += (s[pos + step - 1] < o) ? step : 0;
    const int eq = (pos < u) & (s[pos < 15 ? pos : 15] == o);
    return 2 * pos + eq;
}

// Per-thread bucket counters in LDS, c[bucket][thread] (u16): a thread
// counts its own keys with plain reads and writes, no atomics.  The
// returned value is the key's rank among the thread's earlier keys of the
// same bucket.
template <int NT>
__device__ __forceinline__ uint32_t count_own(uint16_t (*c)[NT], int b, int tid) {
    const uint32_t r = c[b][tid];
    c[b][tid] = static_cast<uint16_t>(r + 1);
    return r;
}

// Plan kernel for a multiway level: per segment (one wave each) a sample of
// up to kMaxSample keys at stratified, hashed positions; its order statistics
// at ranks (j+1)*k/(kSplit+1) become the splitters, duplicates removed.  Also
// writes the equal runs recorded by the previous level.
template <int DT, class V, int NT>
__global__ __launch_bounds__(NT) void k_plan_multi(Args a) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    constexpr int NW = NT / 64;
    static_assert(kMaxSample < 4 * 64, "a lane holds at most four samples");
    __shared__ R s_samp[NW][kMaxSample + 1];
    __shared__ R s_sorted[NW][kMaxSample + 1];

    Ctl* c = a.ctl;
    if (c->error) return;  // an earlier step latched an error: the rest of the call does nothing
    const int p = a.level & 1, q = p ^ 1;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t nseg = static_cast<uint32_t>(c->lc[p].segs);
    reset_next_slot(c, q, nseg, blockIdx.x);
    if (nseg > a.cap_seg) nseg = a.cap_seg;  // an overflow was latched
    const R* src = static_cast<const R*>(p ? a.y_keys : a.x_keys);
    R* ws = s_samp[wv];
    R* so = s_sorted[wv];

    for (uint32_t base = blockIdx.x * NW; base < nseg; base += gridDim.x * NW) {
        const uint32_t si = base + wv;
        const bool valid = si < nseg;
        SegDesc* sd = &a.segs[p][valid ? si : 0];
        int64_t lo = 0, hi = 0, m = 0;
        uint32_t depth = 0;
        int k = 0;
        if (valid) {
            lo = sd->lo;
            hi = sd->hi;
            m = hi - lo;
            depth = sd->depth;
            k = static_cast<int>(m < a.sample_max ? m : a.sample_max);
        }
        for (int i = lane; i < k; i += 64) {
            const int64_t stride = m / k;
            const uint64_t h = mix64((static_cast<uint64_t>(lo) * 0x9e3779b97f4a7c15ull) ^
                                     (static_cast<uint64_t>(hi) << 17) ^ (static_cast<uint64_t>(i) << 40) ^ depth);
            ws[i] = src[lo + i * stride + static_cast<int64_t>(h % static_cast<uint64_t>(stride))];
        }
        __syncthreads();
        // sample ranks (ties broken by sample index) place the sample in
        // order; each lane ranks its up to four samples in one pass over
        // the sample (one LDS read serves four comparisons)
        {
            using O = decltype(K::ord(R()));
            O om[4];
            int rank[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = lane + 64 * r;
                om[r] = i < k ? K::ord(ws[i]) : O(0);
                rank[r] = 0;
            }
#pragma unroll 4
            for (int j = 0; j < k; ++j) {
                const O oj = K::ord(ws[j]);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    rank[r] += (oj < om[r]) | ((oj == om[r]) & (j < lane + 64 * r));
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (lane + 64 * r < k) so[rank[r]] = ws[lane + 64 * r];
        }
        __syncthreads();
        // splitters: the sample's order statistics at ranks (j+1)*k/16, then
        // distinct values only (they come in ascending order)
        uint64_t sj = 0;
        bool keep = false;
        if (lane < kSplit && k > 0) {
            const int idx = ((lane + 1) * k) / (kSplit + 1);
            const int prev = (lane * k) / (kSplit + 1);
            sj = static_cast<uint64_t>(K::ord(so[idx]));
            keep = lane == 0 || sj != static_cast<uint64_t>(K::ord(so[prev]));
        }
        const uint64_t km = __ballot(keep);
        const int u = __popcll(km);
        if (valid) {
            uint64_t* out = a.splitters[p] + static_cast<size_t>(si) * 16;
            if (keep) out[mbcnt(km)] = sj;
            if (lane >= u && lane < 16) out[lane] = ~0ull;
            if (lane < kBStride) a.bcur[static_cast<size_t>(si) * kBStride + lane] = 0;
            if (lane == 0) {
                sd->pad = static_cast<uint32_t>(u);
                sd->cursor = 0;
            }
        }
        __syncthreads();
    }
    run_fills<DT, V, NT>(a, p, blockIdx.x, gridDim.x);
}

// Loads the splitters of segment si into LDS (16 entries, all threads) and
// returns how many are in use.
__device__ __forceinline__ int load_splitters(const Args& a, int p, uint32_t si, uint64_t* s_spl) {
    if (threadIdx.x < 16) s_spl[threadIdx.x] = a.splitters[p][static_cast<size_t>(si) * 16 + threadIdx.x];
    return static_cast<int>(a.segs[p][si].pad);
}

// Per-tile bucket histogram (per-thread counters), then each bucket's
// offset claimed on the segment's bucket cursor.
template <int DT, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_mcount(Args a) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    constexpr int T = NT * EPT;
    static_assert(EPT < 65536, "per-thread counts fit 16 bits");
    __shared__ uint64_t s_spl[16];
    __shared__ uint16_t s_c[kBStride][NT];
    const Ctl* c = a.ctl;
    const int p = a.level & 1;
    uint32_t ntiles = static_cast<uint32_t>(c->lc[p].segs >> 32);
    if (ntiles > a.cap_tile) ntiles = a.cap_tile;  // an overflow was latched
    const uint32_t tile = blockIdx.x;
    if (tile >= ntiles || c->error) return;  // (an error latched by an earlier step: nothing runs)
    const int tid = threadIdx.x;
    const TileDesc td = a.tile_desc[tile];
    const int u = load_splitters(a, p, td.si, s_spl);
#pragma unroll
    for (int b = 0; b < kBStride; ++b) s_c[b][tid] = 0;
    __syncthreads();
    const int64_t tbase = td.lo + static_cast<int64_t>(tile - td.t0) * T;
    const int sl = 0;
    const int el = td.hi < tbase + T ? static_cast<int>(td.hi - tbase) : T;
    const R* tsrc = static_cast<const R*>(p ? a.y_keys : a.x_keys) + tbase;
#pragma unroll 8
    for (int i = 0; i < EPT; ++i) {
        const int off = i * NT + tid;
        if (off >= sl && off < el) count_own<NT>(s_c, bucket_of(static_cast<uint64_t>(K::ord(tsrc[off])), s_spl, u), tid);
    }
    __syncthreads();
    // bucket totals: one wave per group of buckets sums a row of counters;
    // then one thread per bucket claims the tile's offset in the bucket
    __shared__ uint32_t s_tot[kBStride];
    const int lane = tid & 63, wv = tid >> 6;
    for (int b = wv; b < kBStride; b += NT / 64) {
        uint32_t v = 0;
        for (int x = lane; x < NT; x += 64) v += s_c[b][x];
        v = static_cast<uint32_t>(wave_sum(v));
        if (lane == 0) s_tot[b] = v;
    }
    __syncthreads();
    if (tid < kBuckets) {
        const uint32_t v = s_tot[tid];
        uint32_t at = 0;
        if (v) at = atomicAdd(&a.bcur[static_cast<size_t>(td.si) * kBStride + tid], v);
        a.toff[static_cast<size_t>(tile) * kBStride + tid] = at;
    }
}

// Per segment (one wave each): bucket starts from the final bucket cursors
// (the bucket totals), and the next level's lists.  Even buckets are appended
// like the children of the two-way step; odd buckets are final (keys equal to
// a splitter) and, when they sit in the workspace buffer, become equal runs
// written into X by the next level.  The appends of a workgroup's waves take
// one atomic add per list, issued by different threads at once.
template <int DT, int NT>
__global__ __launch_bounds__(NT) void k_mscan(Args a) {
    using K = KeyT<DT>;
    constexpr int NW = NT / 64;
    constexpr int kLists = 2 + kSmallClasses;
    __shared__ unsigned long long s_stat[NW][3];
    __shared__ unsigned long long s_w[NW][kLists];  // per wave: its total of each list's appends
    __shared__ unsigned long long s_base[kLists];   // per list: the workgroup's first slot
    Ctl* c = a.ctl;
    if (c->error) return;  // an earlier step latched an error: the rest of the call does nothing
    const int p = a.level & 1, q = p ^ 1;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t nseg = static_cast<uint32_t>(c->lc[p].segs);
    if (nseg > a.cap_seg) nseg = a.cap_seg;  // an overflow was latched
    const int64_t T = a.tile_keys;
    const int64_t S = a.small_cut;
    unsigned long long fill_keys = 0, next_keys = 0, next_tiles = 0;

    // wave-uniform trip count; waves past the list take part with nothing
    for (uint32_t base = blockIdx.x * NW; base < nseg; base += gridDim.x * NW) {
        const uint32_t si = base + wv;
        const bool valid = si < nseg;
        SegDesc sd{};
        if (valid) sd = a.segs[p][si];
        const int u = static_cast<int>(sd.pad);
        const bool used = valid && lane < 2 * u + 1;
        const uint32_t tot = used ? a.bcur[static_cast<size_t>(si) * kBStride + lane] : 0u;
        const uint32_t start = static_cast<uint32_t>(wave_inclusive_sum(tot, lane)) - tot;
        if (valid && lane < kBStride) a.bstart[static_cast<size_t>(si) * kBStride + lane] = start;
        const int64_t blo = sd.lo + start;
        const int64_t m = tot;
        const bool eqb = (lane & 1) != 0;
        // even bucket: kind 1 partition at L+1, 2 small sort, 0 nothing
        int kind = 0, cls = -1;
        uint32_t nt = 0;
        if (used && !eqb && m > 0) {
            kind = m > S ? 1 : ((m == 1 && q == 0) ? 0 : 2);
            if (kind == 1) nt = seg_tiles(blo, blo + m, T);
            if (kind == 2) cls = small_class(m);
            if (kind == 0) mark_done(a, sd.origin);  // one key, already in X
        }
        if (used && eqb && m > 0 && q == 0) mark_done(a, sd.origin);  // equal keys scattered into X
        // the appends of the whole workgroup, one atomic add per list and
        // workgroup (list 0: segments of level L+1, count | tiles << 32; 1:
        // equal runs, count | chunks << 32; 2 + k: small segments of class k)
        const uint64_t sinc = kind == 1 ? (1ull | (static_cast<uint64_t>(nt) << 32)) : 0ull;
        const bool fill = used && eqb && m > 0 && q == 1;
        const uint32_t nch = fill ? static_cast<uint32_t>((m + kFillChunk - 1) / kFillChunk) : 0u;
        const uint64_t finc = fill ? (1ull | (static_cast<uint64_t>(nch) << 32)) : 0ull;
        const uint64_t sin = wave_inclusive_sum(sinc, lane);
        const uint64_t fin = wave_inclusive_sum(finc, lane);
        if (lane == 63) {
            s_w[wv][0] = sin;
            s_w[wv][1] = fin;
        }
        uint64_t bm_own = 0;
#pragma unroll
        for (int k = 0; k < kSmallClasses; ++k) {
            const uint64_t bm = __ballot(cls == k);
            if (cls == k) bm_own = bm;
            if (lane == 0) s_w[wv][2 + k] = static_cast<unsigned long long>(__popcll(bm));
        }
        __syncthreads();
        if (tid < kLists) {
            unsigned long long total = 0;
            for (int w = 0; w < NW; ++w) total += s_w[w][tid];
            unsigned long long at = 0;
            if (total) {
                if (tid == 0) at = atomicAdd(&c->lc[q].segs, total);
                else if (tid == 1) at = atomicAdd(&c->lc[q].fills, total);
                else at = atomicAdd(&c->lc[q].smalls[tid - 2], static_cast<uint32_t>(total));
            }
            s_base[tid] = at;
        }
        __syncthreads();
        auto wave_base = [&](int list) {
            unsigned long long b = s_base[list];
            for (int w = 0; w < wv; ++w) b += s_w[w][list];
            return b;
        };
        if (kind == 1) {
            const uint64_t at = wave_base(0) + sin - sinc;
            const uint32_t idx = static_cast<uint32_t>(at);
            const uint64_t t0 = at >> 32;
            if (idx >= a.cap_seg || t0 + nt > a.cap_tile) {
                atomicOr(&c->error, ERR_OVERFLOW);
            } else {
                SegDesc d{};
                d.lo = blo;
                d.hi = blo + m;
                d.t0 = static_cast<uint32_t>(t0);
                d.nt = nt;
                d.depth = sd.depth + 1;
                d.origin = sd.origin;
                a.segs[q][idx] = d;
            }
            next_keys += static_cast<unsigned long long>(m);
            next_tiles += nt;
        }
        if (cls >= 0) {
            const uint32_t idx = static_cast<uint32_t>(wave_base(2 + cls)) + mbcnt(bm_own);
            if (idx >= a.cap_small) atomicOr(&c->error, ERR_OVERFLOW);
            else a.smalls[q][static_cast<size_t>(cls) * a.cap_small + idx] = SmallItem{blo, blo + m, sd.origin, 0u};
        }
        // keys equal to a splitter, left in the workspace buffer: written
        // into X by the next level (as the pivot's run of the two-way step)
        if (fill) {
            const uint64_t at = wave_base(1) + fin - finc;
            const uint32_t idx = static_cast<uint32_t>(at);
            if (idx >= a.cap_fill) {
                atomicOr(&c->error, ERR_OVERFLOW);
            } else {
                const uint64_t o = a.splitters[p][static_cast<size_t>(si) * 16 + (lane >> 1)];
                FillItem f;
                f.dst = blo;
                f.len = m;
                f.side = blo;
                f.raw = static_cast<uint64_t>(K::inv(static_cast<decltype(K::ord(typename K::raw()))>(o)));
                f.chunk0 = static_cast<uint32_t>(at >> 32);
                f.origin = sd.origin;
                f.pad1 = 0;
                a.fills[q][idx] = f;
            }
        }
        __syncthreads();  // s_w and s_base are reused by the next round
        if (used && eqb && m > 0) fill_keys += static_cast<unsigned long long>(m);
    }
    // statistics: one set of atomics per workgroup
    fill_keys = wave_sum(fill_keys);
    next_keys = wave_sum(next_keys);
    next_tiles = wave_sum(next_tiles);
    if (lane == 0) {
        s_stat[wv][0] = fill_keys;
        s_stat[wv][1] = next_keys;
        s_stat[wv][2] = next_tiles;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long f = 0, k = 0, t = 0;
        for (int w = 0; w < NW; ++w) {
            f += s_stat[w][0];
            k += s_stat[w][1];
            t += s_stat[w][2];
        }
        if (f) atomicAdd(&c->fill_keys, f);
        if (k) {
            atomicAdd(&c->part_keys, k);
            atomicAdd(&c->lc[q].keys, k);
            atomicAdd(&c->level_keys[level_slot(a.level + 1)], k);
        }
        if (t) atomicAdd(&c->tiles, t);
    }
}

// Per tile: keys staged in LDS in bucket order (a key's rank in its bucket
// from one LDS counter per bucket, its position that rank past the bucket's
// start in the tile), then every bucket's run copied out coalesced to its
// place in the other buffer.
template <int DT, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_mscatter(Args a) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    constexpr int T = NT * EPT;
    __shared__ uint64_t s_spl[16];
    __shared__ R s_k[T];
    __shared__ uint8_t s_b[T];
    __shared__ uint32_t s_cnt[kBStride], s_start[kBStride], s_off[kBStride];
    const Ctl* c = a.ctl;
    const int p = a.level & 1;
    uint32_t ntiles = static_cast<uint32_t>(c->lc[p].segs >> 32);
    if (ntiles > a.cap_tile) ntiles = a.cap_tile;  // an overflow was latched
    const uint32_t tile = blockIdx.x;
    if (tile >= ntiles || c->error) return;  // (an error latched by an earlier step: nothing runs)
    const int tid = threadIdx.x, lane = tid & 63;
    const TileDesc td = a.tile_desc[tile];
    const int u = load_splitters(a, p, td.si, s_spl);
    if (tid < kBStride) {
        s_cnt[tid] = 0;
        s_off[tid] = a.bstart[static_cast<size_t>(td.si) * kBStride + tid] +
                     a.toff[static_cast<size_t>(tile) * kBStride + tid];
    }
    __syncthreads();
    const int64_t tbase = td.lo + static_cast<int64_t>(tile - td.t0) * T;
    const int sl = 0;
    const int el = td.hi < tbase + T ? static_cast<int>(td.hi - tbase) : T;
    const R* tsrc = static_cast<const R*>(p ? a.y_keys : a.x_keys) + tbase;
    R* dst = static_cast<R*>(p ? a.x_keys : a.y_keys) + td.lo;
    R key[EPT];
    uint32_t br[EPT];  // bucket | rank of the key among the tile's keys of that bucket << 8
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int off = i * NT + tid;
        const bool ok = off >= sl && off < el;
        key[i] = ok ? tsrc[off] : R(0);
        const uint32_t b = ok ? static_cast<uint32_t>(bucket_of(static_cast<uint64_t>(K::ord(key[i])), s_spl, u))
                              : 0xffu;
        br[i] = ok ? (b | (atomicAdd(&s_cnt[b], 1u) << 8)) : 0xffu;
    }
    __syncthreads();
    if (tid < 64) {
        // exclusive scan of the tile's bucket counts (one wave)
        const uint32_t v = lane < kBStride ? s_cnt[lane] : 0u;
        const uint32_t inc = static_cast<uint32_t>(wave_inclusive_sum(v, lane));
        if (lane < kBStride) s_start[lane] = inc - v;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const uint32_t b = br[i] & 0xffu;
        if (b != 0xffu) {
            const uint32_t pos = s_start[b] + (br[i] >> 8);
            s_k[pos] = key[i];
            s_b[pos] = static_cast<uint8_t>(b);
        }
    }
    __syncthreads();
    const int cnt = el - sl;
    for (int x = tid; x < cnt; x += NT) {
        const int b = s_b[x];
        __builtin_nontemporal_store(s_k[x], dst + s_off[b] + (x - static_cast<int>(s_start[b])));  // streaming
    }
}

}  // namespace bqs
