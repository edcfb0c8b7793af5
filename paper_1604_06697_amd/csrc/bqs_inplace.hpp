// In-place partition step (Section 3, Algorithm 3, and Section 3.2).
//
// The default step partitions out of place, into a second buffer of n keys
// (and payloads).  This step keeps keys and payloads in the caller's
// buffers, as Algorithm 3 does, with a workspace of one bit per key plus
// per-tile counts.  Algorithm 3 records, block by block, the offsets of the
// elements that sit on the wrong side of the pivot (its two offset buffers)
// and then swaps them in pairs, the k-th wrong element from the left with
// the k-th wrong element from the right.  Here the recording covers a whole
// level at once and the pairs are swapped in parallel.  Per level, for each
// segment [lo, hi) with pivot p (tiles of kIpT keys, tile j covering
// [lo + j*kIpT, +kIpT) clipped to the segment):
//   count    one workgroup per tile: each key's class as one bit -- class L
//            is x < p, or x <= p in a segment whose pivot was fixed by its
//            parent -- and the tile's class-L keys and keys equal to p;
//   scan     one workgroup per segment: the boundary b = lo + (class-L
//            keys).  Left of b a key is misplaced when it is not class L,
//            right of b when it is; both sides hold the same number M of
//            them.  Per tile: its misplaced keys on each side and running
//            sums that rank the misplaced keys left of b from the left end
//            and those right of b from the right end;
//   exchange the misplaced key of rank k on the left and the one of rank k
//            on the right change places.  The tiles of the larger side own
//            the exchange: a workgroup takes one such tile with misplaced
//            keys, stages it in LDS, finds its partners' tiles by binary
//            search over the running sums and their positions by the
//            class bits, and writes each moved key once -- the point of the
//            cyclic permutation of Section 3.2, where no element passes
//            through a temporary twice.  Every position is written by one
//            workgroup only, the class bits never change during the step,
//            and the result does not depend on scheduling;
//   complete one thread per segment: children [lo, b) and [b, hi).
//
// Equal keys.  With classes x < p the right child holds every key equal
// to p.  When they are many (at least an eighth of the child), or when the
// left child is empty, the right child is partitioned next with the same
// pivot and classes x <= p: p is its smallest key, so its left part holds
// exactly the keys equal to p and is finished.  Every segment therefore
// shrinks by at least one key within two levels (p is a key of the
// segment), and a segment of equal keys takes two count passes and no
// exchange.
#pragma once

namespace bqs {

// Bits [lo, hi) of a 64-bit word, 0 <= lo <= hi <= 64.
__device__ __forceinline__ uint64_t bits_between(int lo, int hi) {
    const uint64_t up = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    const uint64_t down = lo >= 64 ? ~0ull : ((1ull << lo) - 1ull);
    return up & ~down;
}

// The misplaced keys among the 64 of class word `w` of a tile, for a part
// [s0, s1) of the tile (tile offsets) on side `side` (0: left of the
// boundary, where keys not in class L are misplaced; 1: right of it).
__device__ __forceinline__ uint64_t misplaced_bits(uint64_t word, int w, int s0, int s1, int side) {
    const int b0 = s0 - 64 * w, b1 = s1 - 64 * w;
    const int lo = b0 < 0 ? 0 : (b0 > 64 ? 64 : b0);
    const int hi = b1 < 0 ? 0 : (b1 > 64 ? 64 : b1);
    if (hi <= lo) return 0ull;
    return (side == 0 ? ~word : word) & bits_between(lo, hi);
}

// The part of a tile at offset `tlo` (of `len` keys) on side `side` of the
// boundary b: tile offsets [s0, s1).
__device__ __forceinline__ void side_part(int64_t tlo, int len, int64_t b, int side, int& s0, int& s1) {
    const int64_t k = b - tlo;
    const int cut = k < 0 ? 0 : (k > len ? len : static_cast<int>(k));
    s0 = side == 0 ? 0 : cut;
    s1 = side == 0 ? cut : len;
}

// ------------------------------------------------------------------ count --

template <int DT, int NT, int EPT>
__device__ void ip_count_tile(const Args& a, int p, uint32_t t, uint32_t* s_red) {
    using K = KeyT<DT>;
    using R = typename K::raw;
    constexpr int T = NT * EPT;
    constexpr int NW = NT / 64;
    static_assert(T == kIpT, "in-place tile size");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const TileDesc td = a.tile_desc[t];
    const bool le = (a.segs[p][td.si].pad & kSegForced) != 0;
    const int64_t tlo = td.lo + static_cast<int64_t>(t - td.t0) * T;
    const int len = static_cast<int>(td.hi - tlo < T ? td.hi - tlo : T);
    const R* src = static_cast<const R*>(a.x_keys) + tlo;
    R raw[EPT];
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int o = r * NT + tid;
        raw[r] = src[o < len ? o : len - 1];
    }
    uint64_t* mw = a.ipmask + static_cast<size_t>(t) * kIpWords;
    uint32_t nl = 0, ne = 0;
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int o = r * NT + tid;
        const bool valid = o < len;
        const uint64_t x = static_cast<uint64_t>(K::ord(raw[r]));
        const uint64_t bl = __ballot(valid && (le ? x <= td.pivot : x < td.pivot));
        const uint64_t be = __ballot(valid && x == td.pivot);
        if (lane == 0) mw[r * NW + wv] = bl;
        nl += static_cast<uint32_t>(__popcll(bl));
        ne += static_cast<uint32_t>(__popcll(be));
    }
    if (lane == 0) {
        s_red[wv] = nl;
        s_red[NW + wv] = ne;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t snl = 0, sne = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            snl += s_red[w];
            sne += s_red[NW + w];
        }
        a.iptile[t].nl = snl;
        a.iptile[t].neq = sne;
    }
    __syncthreads();  // s_red is free again
}

template <int DT, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_ip_count(Args a) {
    __shared__ uint32_t s_red[2 * (NT / 64)];
    const Ctl* c = a.ctl;
    const int p = a.level & 1;
    uint32_t ntiles = static_cast<uint32_t>(c->lc[p].segs >> 32);
    if (ntiles > a.cap_tile) ntiles = a.cap_tile;
    if (c->error) return;  // an earlier step latched an error: the rest of the call does nothing
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) ip_count_tile<DT, NT, EPT>(a, p, t, s_red);
}

// ------------------------------------------------------------------- scan --

// Exclusive prefix sum over the workgroup (NT threads, one value each) and
// the workgroup total.  s_w: NT/64 words of LDS.
template <int NT>
__device__ __forceinline__ uint64_t block_exclusive_sum(uint64_t v, uint64_t* s_w, uint64_t& total) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t inc = wave_inclusive_sum(v, lane);
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint64_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        before += w < wv ? s_w[w] : 0u;
        total += s_w[w];
    }
    __syncthreads();  // s_w is free again
    return before + inc - v;
}

// Class-L keys of tile (t0 + j) of a segment left of the boundary b.
__device__ __forceinline__ uint32_t class_left_of(const Args& a, uint32_t t, int k) {
    const uint64_t* mw = a.ipmask + static_cast<size_t>(t) * kIpWords;
    uint32_t left = 0;
    for (int w = 0; w < (k >> 6); ++w) left += static_cast<uint32_t>(__popcll(mw[w]));
    if (k & 63) left += static_cast<uint32_t>(__popcll(mw[k >> 6] & bits_between(0, k & 63)));
    return left;
}

// One segment of an in-place level, by all NT threads of a workgroup, in
// three passes over its tiles (TPT consecutive tiles per thread and pass):
// (1) its class-L keys and keys equal to the pivot, hence the boundary;
// (2) per tile the misplaced keys on each side and the ranks of the first
// ones from the left end (left side) and, for now, the running sum from the
// left (right side); (3) the right-side ranks counted from the right end,
// the segment's values in every tile, and the rank table of the partner
// side.
template <int NT>
__device__ void ip_scan_segment(const Args& a, int p, uint32_t si, uint64_t* s_w) {
    constexpr int TPT = 8;
    constexpr uint32_t CH = NT * TPT;
    const int tid = threadIdx.x;
    SegDesc* sd = &a.segs[p][si];
    const int64_t lo = sd->lo, hi = sd->hi;
    const uint32_t t0 = sd->t0, nt = sd->nt;
    __shared__ uint32_t s_tbase;
    // (1)
    uint64_t nl = 0, ne = 0;
    for (uint32_t j = tid; j < nt; j += NT) {
        nl += a.iptile[t0 + j].nl;
        ne += a.iptile[t0 + j].neq;
    }
    uint64_t tot = 0;
    (void)block_exclusive_sum<NT>((nl << 32) | ne, s_w, tot);
    nl = tot >> 32;
    ne = tot & 0xffffffffull;
    const int64_t b = lo + static_cast<int64_t>(nl);
    const bool aright = b - lo < hi - b;  // the right part is the larger one
    // (2)
    uint64_t carry = 0;  // misplaced so far: left side << 32 | right side
    for (uint32_t jb = 0; jb < nt; jb += CH) {
        const uint32_t j0 = jb + static_cast<uint32_t>(tid) * TPT;
        uint32_t ml[TPT], mr[TPT];
        uint64_t mine = 0;
#pragma unroll
        for (int i = 0; i < TPT; ++i) {
            const uint32_t j = j0 + i;
            ml[i] = mr[i] = 0;
            if (j < nt) {
                const int64_t tlo = lo + static_cast<int64_t>(j) * kIpT;
                const int64_t thi = hi - tlo < kIpT ? hi : tlo + kIpT;
                const uint32_t tnl = a.iptile[t0 + j].nl;
                if (thi <= b) {
                    ml[i] = static_cast<uint32_t>(thi - tlo) - tnl;
                } else if (tlo >= b) {
                    mr[i] = tnl;
                } else {
                    const int k = static_cast<int>(b - tlo);
                    const uint32_t left = class_left_of(a, t0 + j, k);
                    ml[i] = static_cast<uint32_t>(k) - left;
                    mr[i] = tnl - left;
                }
                mine += (static_cast<uint64_t>(ml[i]) << 32) | mr[i];
            }
        }
        uint64_t ctot = 0;
        uint64_t run = carry + block_exclusive_sum<NT>(mine, s_w, ctot);
#pragma unroll
        for (int i = 0; i < TPT; ++i) {
            const uint32_t j = j0 + i;
            if (j < nt) {
                IpTile& it = a.iptile[t0 + j];
                it.mis[0] = ml[i];
                it.mis[1] = mr[i];
                it.rank[0] = static_cast<uint32_t>(run >> 32);
                run += (static_cast<uint64_t>(ml[i]) << 32) | mr[i];
                it.rank[1] = static_cast<uint32_t>(run);  // inclusive, from the left: converted in (3)
            }
        }
        carry += ctot;
    }
    const uint32_t M = static_cast<uint32_t>(carry);  // == carry >> 32
    if (tid == 0) {
        if ((carry >> 32) != (carry & 0xffffffffull)) atomicOr(&a.ctl->error, ERR_OVERFLOW);  // inconsistent
        const uint32_t entries = (M + kIpRankStep - 1) / kIpRankStep;
        uint32_t tb = atomicAdd(&a.ctl->lc[p].tab, entries);
        if (tb + entries > a.cap_tab) {
            atomicOr(&a.ctl->error, ERR_OVERFLOW);
            tb = 0;
        }
        s_tbase = tb;
        sd->cursor = nl | (ne << 32);
        sd->pad = (sd->pad & kSegForced) | (aright ? kSegARight : 0u);
    }
    __syncthreads();
    const uint32_t tbase = s_tbase;
    const int bside = aright ? 0 : 1;  // the partner side: the smaller part
    // (3)
    for (uint32_t j = tid; j < nt; j += NT) {
        IpTile& it = a.iptile[t0 + j];
        const uint32_t r1 = M - it.rank[1];
        it.rank[1] = r1;
        it.seg_nl = static_cast<uint32_t>(nl);
        it.flags = aright ? kSegARight : 0u;
        it.tbase = tbase;
        // partner-side tiles: entry e names the tile of rank e * step
        const uint32_t rb = bside == 0 ? it.rank[0] : r1;
        const uint32_t m = it.mis[bside];
        for (uint32_t e = (rb + kIpRankStep - 1) / kIpRankStep; e * kIpRankStep < rb + m; ++e)
            if (tbase + e < a.cap_tab) a.iprank[tbase + e] = t0 + j;
    }
    __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void k_ip_scan(Args a) {
    __shared__ uint64_t s_w[NT / 64];
    const Ctl* c = a.ctl;
    if (c->error) return;  // an earlier step latched an error: the rest of the call does nothing
    const int p = a.level & 1;
    uint32_t nseg = static_cast<uint32_t>(c->lc[p].segs);
    if (nseg > a.cap_seg) nseg = a.cap_seg;
    for (uint32_t si = blockIdx.x; si < nseg; si += gridDim.x) ip_scan_segment<NT>(a, p, si, s_w);
}

// --------------------------------------------------------------- exchange --

template <int DT, class V, int NT, int EPT>
struct IpLds {
    using R = typename KeyT<DT>::raw;
    using VS = typename ValStore<V>::type;
    static constexpr bool HV = !std::is_same<V, NoVal>::value;
    static constexpr int T = NT * EPT;
    R k[T];                  // the owning tile's part, by tile offset
    VS v[HV ? T : 1];
    uint16_t pos[T];         // tile offset of the owned misplaced key of local rank i
};

// The class words of tile t seen by one wave: lane w holds word w, its
// misplaced bits for part [s0, s1) on side `side`, and the misplaced keys
// of the words before it in rank order (ascending offsets on the left side,
// descending on the right side).
struct IpWords {
    uint64_t bits;
    uint32_t before;
};

__device__ __forceinline__ IpWords ip_words(const Args& a, uint32_t t, int s0, int s1, int side, int lane) {
    static_assert(kIpWords == 64, "one class word per lane");
    IpWords r;
    const uint64_t word = a.ipmask[static_cast<size_t>(t) * kIpWords + lane];
    r.bits = misplaced_bits(word, lane, s0, s1, side);
    const uint64_t c = static_cast<uint64_t>(__popcll(r.bits));
    const uint64_t inc = wave_inclusive_sum(c, lane);
    const uint64_t tot = bcast64(inc, 63);
    r.before = static_cast<uint32_t>(side == 0 ? inc - c : tot - inc);
    return r;
}

// Misplaced keys of word w that precede lane `lane` in rank order.
__device__ __forceinline__ uint32_t ip_rank_in_word(uint64_t m, int lane, int side) {
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t above = lane == 63 ? 0ull : (~0ull << (lane + 1));
    return static_cast<uint32_t>(__popcll(m & (side == 0 ? below : above)));
}

template <int DT, class V, int NT, int EPT>
__device__ void ip_exchange_tile(const Args& a, uint32_t t, IpLds<DT, V, NT, EPT>& L) {
    using R = typename KeyT<DT>::raw;
    using VS = typename ValStore<V>::type;
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    constexpr int T = NT * EPT;
    constexpr int NW = NT / 64;
    // opaque: keeps the per-item offsets and lane masks from being hoisted
    // out of the caller's loop over tiles (and spilled across it)
    const int tid = opaque(static_cast<int>(threadIdx.x)), lane = tid & 63, wv = tid >> 6;
    // (fields picked with selects: an array member indexed at run time
    // would put the copy in scratch memory)
    const IpTile me = a.iptile[t];
    const int aside = (me.flags & kSegARight) ? 1 : 0, bside = 1 - aside;
    const uint32_t c = aside ? me.mis[1] : me.mis[0];
    if (c == 0) return;
    const TileDesc td = a.tile_desc[t];
    const int64_t b = td.lo + static_cast<int64_t>(me.seg_nl);
    const uint32_t base = aside ? me.rank[1] : me.rank[0];
    const uint32_t nt = seg_tiles(td.lo, td.hi, T);
    const int64_t tlo = td.lo + static_cast<int64_t>(t - td.t0) * T;
    const int len = static_cast<int>(td.hi - tlo < T ? td.hi - tlo : T);
    int s0, s1;
    side_part(tlo, len, b, aside, s0, s1);
    // tile base pointers (uniform): per-item addresses are 32-bit offsets
    R* const tk = static_cast<R*>(a.x_keys) + tlo;
    VS* const tv = static_cast<VS*>(a.x_vals) + (HV ? tlo : 0);

    // 1. the owning tile's part into LDS; the offset of each owned
    // misplaced key by its rank.  The loads are issued first, so that they
    // overlap the lookup of the first partner tile.
    R own_k[EPT];
    VS own_v[HV ? EPT : 1];
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int o = r * NT + tid;
        if (o >= s0 && o < s1) {
            own_k[r] = tk[o];
            if constexpr (HV) own_v[r] = tv[o];
        }
    }
    const IpWords wd = ip_words(a, t, s0, s1, aside, lane);
    // first partner tile: the table names the tile holding rank
    // floor(base / step) * step; walk on in rank order to the one holding base
    uint32_t u = a.iprank[me.tbase + base / kIpRankStep];
    for (;;) {
        const IpTile ut = a.iptile[u];
        if (base < (bside ? ut.rank[1] + ut.mis[1] : ut.rank[0] + ut.mis[0])) break;
        u = bside == 0 ? u + 1 : u - 1;
        if (u < td.t0 || u >= td.t0 + nt) break;  // inconsistent ranks (caught below)
    }
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int o = r * NT + tid;
        if (o >= s0 && o < s1) {
            L.k[o] = own_k[r];
            if constexpr (HV) L.v[o] = own_v[r];
        }
        const int w = r * NW + wv;
        const uint64_t m = bcast64(wd.bits, w);
        const uint32_t before = static_cast<uint32_t>(__shfl(static_cast<int>(wd.before), w, 64));
        if ((m >> lane) & 1ull)
            L.pos[before + ip_rank_in_word(m, lane, aside)] = static_cast<uint16_t>(o);
    }
    __syncthreads();

    // 2. partner tiles in rank order; each swaps its share of ranks
    // [base, base + c) with the owned keys through LDS
    uint32_t covered = 0;
    while (covered < c) {
        if (u < td.t0 || u >= td.t0 + nt) {
            if (tid == 0) atomicOr(&a.ctl->error, ERR_OVERFLOW);  // inconsistent ranks
            break;
        }
        const IpTile ut = a.iptile[u];
        const uint32_t ub = bside ? ut.rank[1] : ut.rank[0], um = bside ? ut.mis[1] : ut.mis[0];
        const uint32_t r0 = ub > base ? ub : base;
        const uint32_t r1 = ub + um < base + c ? ub + um : base + c;
        if (r1 > r0) {
            const int64_t ulo = td.lo + static_cast<int64_t>(u - td.t0) * T;
            const int ulen = static_cast<int>(td.hi - ulo < T ? td.hi - ulo : T);
            int q0, q1;
            side_part(ulo, ulen, b, bside, q0, q1);
            const IpWords wd = ip_words(a, u, q0, q1, bside, lane);
            R* const uk = static_cast<R*>(a.x_keys) + ulo;
            VS* const uv = static_cast<VS*>(a.x_vals) + (HV ? ulo : 0);
            // a key is this workgroup's if it is a partner (rank in [r0, r1))
            // or lies between two of them: counted in rank order, the
            // misplaced keys before it number between lr0 and lr1.  Only
            // two bit masks live across the loads; the ranks are recomputed
            // for the swaps.
            const uint32_t lr0 = r0 - ub, lr1 = r1 - ub;
            auto before_of = [&](int r, uint64_t& m) -> uint32_t {
                const int w = r * NW + wv;
                m = bcast64(wd.bits, w);
                return static_cast<uint32_t>(__shfl(static_cast<int>(wd.before), w, 64)) +
                       ip_rank_in_word(m, lane, bside);
            };
            uint32_t own = 0, hit = 0;
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                uint64_t m;
                const uint32_t before = before_of(r, m);
                const int o = r * NT + tid;
                const bool mis = (m >> lane) & 1ull;
                const bool h = mis && before >= lr0 && before < lr1;
                const bool in = o >= q0 && o < q1 && (h || (!mis && before > lr0 && before < lr1));
                hit |= h ? 1u << r : 0u;
                own |= in ? 1u << r : 0u;
            }
            R x[EPT];
#pragma unroll
            for (int r = 0; r < EPT; ++r)
                if ((own >> r) & 1u) x[r] = uk[r * NT + tid];
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                // (the shuffles run with every lane active: a lane outside
                // the branch could not serve as a source)
                uint64_t m;
                const uint32_t bf = before_of(r, m);
                if ((hit >> r) & 1u) {
                    const int op = L.pos[ub + bf - base];
                    const R x_own = L.k[op];
                    L.k[op] = x[r];
                    x[r] = x_own;
                }
                if ((own >> r) & 1u) uk[r * NT + tid] = x[r];
            }
            if constexpr (HV) {
                // payloads follow with the same masks (a second pass keeps
                // the key registers free)
                VS y[EPT];
#pragma unroll
                for (int r = 0; r < EPT; ++r)
                    if ((own >> r) & 1u) y[r] = uv[r * NT + tid];
#pragma unroll
                for (int r = 0; r < EPT; ++r) {
                    uint64_t m;
                    const uint32_t bf = before_of(r, m);
                    if ((hit >> r) & 1u) {
                        const int op = L.pos[ub + bf - base];
                        const VS y_own = L.v[op];
                        L.v[op] = y[r];
                        y[r] = y_own;
                    }
                    if ((own >> r) & 1u) uv[r * NT + tid] = y[r];
                }
            }
            covered += r1 - r0;
        }
        u = bside == 0 ? u + 1 : u - 1;
    }
    __syncthreads();
    // 3. the owning tile's part back in place
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int o = r * NT + tid;
        if (o >= s0 && o < s1) {
            tk[o] = L.k[o];
            if constexpr (HV) tv[o] = L.v[o];
        }
    }
    __syncthreads();  // LDS is free for the next tile
}

// At most 168 VGPRs: three waves per SIMD (no spills).
template <int DT, class V, int NT, int EPT>
__global__ __launch_bounds__(NT, 3) void k_ip_exchange(Args a) {
    __shared__ IpLds<DT, V, NT, EPT> s_lds;
    const Ctl* c = a.ctl;
    const int p = a.level & 1;
    uint32_t ntiles = static_cast<uint32_t>(c->lc[p].segs >> 32);
    if (ntiles > a.cap_tile) ntiles = a.cap_tile;
    if (c->error) return;  // an earlier step latched an error: the rest of the call does nothing
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) ip_exchange_tile<DT, V, NT, EPT>(a, t, s_lds);
}

// --------------------------------------------------------------- complete --

// Children of every in-place segment of level L (one thread per segment):
// [lo, b) and [b, hi), see the comment at the top of this file.
__device__ inline void ip_complete_body(const Args& a, int level, uint32_t bid, uint32_t nblk) {
    constexpr uint32_t WG = 256;
    Ctl* c = a.ctl;
    const int p = level & 1, q = p ^ 1;
    const int lane = lane_id();
    uint32_t nseg = static_cast<uint32_t>(c->lc[p].segs);
    if (nseg > a.cap_seg) nseg = a.cap_seg;  // an overflow was latched
    const int64_t T = kIpT;
    const int64_t S = a.small_cut;
    unsigned long long next_keys = 0, next_tiles = 0;
    for (uint32_t base = bid * WG; base < nseg; base += nblk * WG) {
        const uint32_t si = base + threadIdx.x;
        const bool valid = si < nseg;
        int64_t clo[2] = {0, 0}, chi[2] = {0, 0};
        bool forced[2] = {false, false};
        uint32_t depth = 0, origin = 0;
        uint64_t pv = 0, praw = 0;
        bool dropped = false;  // a part of equal keys that is finished
        if (valid) {
            const SegDesc sd = a.segs[p][si];
            origin = sd.origin;
            const int64_t nl = static_cast<int64_t>(sd.cursor & 0xffffffffull);
            const int64_t ne = static_cast<int64_t>(sd.cursor >> 32);
            const int64_t b = sd.lo + nl;
            depth = sd.depth + 1;
            pv = sd.pivot;
            praw = sd.pivot_raw;
            if (nl > sd.hi - sd.lo || ne > sd.hi - sd.lo) {
                atomicOr(&c->error, ERR_OVERFLOW);
            } else if (sd.pad & kSegForced) {
                // left part: the keys equal to the pivot, finished
                clo[1] = b;
                chi[1] = sd.hi;
                dropped = b > sd.lo;
            } else {
                clo[0] = sd.lo;
                chi[0] = b;
                const int64_t right = sd.hi - b;
                if (right > ne) {  // not all equal to the pivot
                    clo[1] = b;
                    chi[1] = sd.hi;
                    forced[1] = ne > 0 && (nl == 0 || 8 * ne >= right);
                } else {
                    dropped = right > 0;
                }
            }
        }
        if (dropped) mark_done(a, origin);
        int kind[2], cls[2];
        uint32_t nt[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t m = chi[h] - clo[h];
            kind[h] = m <= 1 ? 0 : (m > S ? 1 : 2);
            nt[h] = kind[h] == 1 ? seg_tiles(clo[h], chi[h], T) : 0u;
            cls[h] = kind[h] == 2 ? small_class(m) : -1;
            if (m == 1) mark_done(a, origin);  // one key, in place
        }
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
                    if (forced[h]) {
                        d.pad = kSegForced;
                        d.pivot = pv;
                        d.pivot_raw = praw;
                    }
                    a.segs[q][idx] = d;
                }
                ++idx;
                t0 += nt[h];
                next_keys += static_cast<unsigned long long>(chi[h] - clo[h]);
                next_tiles += nt[h];
            }
        }
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
    }
    next_keys = wave_sum(next_keys);
    next_tiles = wave_sum(next_tiles);
    if (lane == 0) {
        if (next_keys) {
            atomicAdd(&c->part_keys, next_keys);
            atomicAdd(&c->lc[q].keys, next_keys);
            atomicAdd(&c->level_keys[level_slot(level + 1)], next_keys);
        }
        if (next_tiles) atomicAdd(&c->tiles, next_tiles);
    }
}

template <class V>
__global__ __launch_bounds__(256) void k_ip_complete(Args a) {
    if (a.ctl->error) return;  // an earlier step latched an error: the rest of the call does nothing
    ip_complete_body(a, a.level, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------- tail --

// The in-place levels from a.level on, by one workgroup of NT threads: the
// rest of an in-place sort whose enqueued levels did not reach the end.
template <int DT, class V, int NT, int EPT, int SP>
struct IpTailLds {
    static constexpr size_t mx(size_t x, size_t y) { return x > y ? x : y; }
    static constexpr size_t bytes =
        mx(mx(sizeof(IpLds<DT, V, NT, EPT>), sizeof(PlanLds<DT, NT>)), sizeof(BucketLds<DT, V, NT, SP>));
};

// Barrier of the tail's steps: the steps hand data to each other through
// global memory (lists, counts, class bits, keys), written with plain
// stores and atomics by any wave of the workgroup.
__device__ __forceinline__ void tail_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ unsigned tail_error(const Ctl* c) {
    return __hip_atomic_load(&c->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DT, class V, int NT, int EPT, int SP>
__global__ __launch_bounds__(NT) void k_ip_tail(Args a) {
    static_assert(NT == 256, "the plan and completion steps run 256 threads");
    using TL = IpTailLds<DT, V, NT, EPT, SP>;
    __shared__ alignas(16) unsigned char s_raw[TL::bytes];
    __shared__ uint32_t s_red[2 * (NT / 64)];
    __shared__ uint64_t s_w[NT / 64];
    Ctl* c = a.ctl;
    if (tail_error(c)) return;  // an earlier step latched an error: the rest of the call does nothing
    const int level_cap = 4 * a.depth_limit + 64;
    for (int L = a.level;; ++L) {
        const int p = L & 1;
        const unsigned long long sc =
            __hip_atomic_load(&c->lc[p].segs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t nseg = static_cast<uint32_t>(sc);
        uint32_t ntile = static_cast<uint32_t>(sc >> 32);
        if (nseg > a.cap_seg) nseg = a.cap_seg;
        if (ntile > a.cap_tile) ntile = a.cap_tile;
        plan_body<DT, V, NT>(a, L, 0, 1, *reinterpret_cast<PlanLds<DT, NT>*>(s_raw));
        tail_sync();
        small_all_body<DT, V, NT, SP>(a, L, 0, 1, *reinterpret_cast<BucketLds<DT, V, NT, SP>*>(s_raw));
        tail_sync();
        if (nseg == 0 || tail_error(c)) break;
        if (L >= level_cap) {
            if (threadIdx.x == 0) atomicOr(&c->error, ERR_OVERFLOW);
            break;
        }
        for (uint32_t t = 0; t < ntile; ++t) ip_count_tile<DT, NT, EPT>(a, p, t, s_red);
        tail_sync();
        for (uint32_t si = 0; si < nseg; ++si) ip_scan_segment<NT>(a, p, si, s_w);
        tail_sync();
        if (tail_error(c)) break;
        auto& xl = *reinterpret_cast<IpLds<DT, V, NT, EPT>*>(s_raw);
        for (uint32_t t = 0; t < ntile; ++t) ip_exchange_tile<DT, V, NT, EPT>(a, t, xl);
        tail_sync();
        ip_complete_body(a, L, 0, 1);
        tail_sync();
    }
}

}  // namespace bqs
