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
    if (blockIdx.x >= ntiles || c->error) return;  // (an error latched by an earlier step: nothing runs)
    ip_count_tile<DT, NT, EPT>(a, p, blockIdx.x, s_red);
}

// ------------------------------------------------------------------- scan --

// Exclusive prefix sum over the workgroup (NT threads, one value each) and
// the workgroup total.  s_w: NT/64 words of LDS.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t* s_w, uint32_t& total) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t inc = static_cast<uint32_t>(wave_inclusive_sum(static_cast<uint64_t>(v), lane));
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        before += w < wv ? s_w[w] : 0u;
        total += s_w[w];
    }
    __syncthreads();  // s_w is free again
    return before + inc - v;
}

template <int NT>
__device__ void ip_scan_segment(const Args& a, int p, uint32_t si, uint32_t* s_w) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    SegDesc* sd = &a.segs[p][si];
    const int64_t lo = sd->lo, hi = sd->hi;
    const uint32_t t0 = sd->t0, nt = sd->nt;
    // class-L keys and keys equal to the pivot
    uint64_t nl = 0, ne = 0;
    for (uint32_t j = tid; j < nt; j += NT) {
        nl += a.iptile[t0 + j].nl;
        ne += a.iptile[t0 + j].neq;
    }
    nl = wave_sum(nl);
    ne = wave_sum(ne);
    __shared__ unsigned long long s_tot[2][NW];
    if ((tid & 63) == 0) {
        s_tot[0][tid >> 6] = nl;
        s_tot[1][tid >> 6] = ne;
    }
    __syncthreads();
    nl = ne = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        nl += s_tot[0][w];
        ne += s_tot[1][w];
    }
    __syncthreads();
    const int64_t b = lo + static_cast<int64_t>(nl);
    // misplaced keys per tile and side, with running sums
    uint32_t carry_l = 0, carry_r = 0;
    for (uint32_t jb = 0; jb < nt; jb += NT) {
        const uint32_t j = jb + tid;
        uint32_t mis_l = 0, mis_r = 0;
        if (j < nt) {
            const int64_t tlo = lo + static_cast<int64_t>(j) * kIpT;
            const int64_t thi = hi - tlo < kIpT ? hi : tlo + kIpT;
            const uint32_t tnl = a.iptile[t0 + j].nl;
            if (thi <= b) {
                mis_l = static_cast<uint32_t>(thi - tlo) - tnl;
            } else if (tlo >= b) {
                mis_r = tnl;
            } else {
                // the tile holding the boundary: class-L keys left of it
                const int k = static_cast<int>(b - tlo);
                const uint64_t* mw = a.ipmask + static_cast<size_t>(t0 + j) * kIpWords;
                uint32_t left = 0;
                for (int w = 0; w < (k >> 6); ++w) left += static_cast<uint32_t>(__popcll(mw[w]));
                if (k & 63) left += static_cast<uint32_t>(__popcll(mw[k >> 6] & bits_between(0, k & 63)));
                mis_l = static_cast<uint32_t>(k) - left;
                mis_r = tnl - left;
            }
        }
        uint32_t tot_l = 0, tot_r = 0;
        const uint32_t ex_l = block_exclusive_sum<NT>(mis_l, s_w, tot_l);
        const uint32_t ex_r = block_exclusive_sum<NT>(mis_r, s_w, tot_r);
        if (j < nt) {
            IpTile& it = a.iptile[t0 + j];
            it.mis[0] = mis_l;
            it.mis[1] = mis_r;
            it.rank[0] = carry_l + ex_l;
            it.rank[1] = carry_r + ex_r + mis_r;
        }
        carry_l += tot_l;
        carry_r += tot_r;
    }
    if (tid == 0) {
        if (carry_l != carry_r) atomicOr(&a.ctl->error, ERR_OVERFLOW);  // inconsistent counts
        sd->cursor = static_cast<unsigned long long>(nl) | (static_cast<unsigned long long>(ne) << 32);
        sd->pad = (sd->pad & kSegForced) | (b - lo < hi - b ? kSegARight : 0u);
    }
    __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void k_ip_scan(Args a) {
    __shared__ uint32_t s_w[NT / 64];
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
    uint32_t wpre[T / 64];   // per class word: misplaced keys in the words before it (in rank order)
    uint32_t omin, omax;     // offsets of a partner tile that this workgroup owns
    uint32_t u;              // first partner tile
};

// Per class word w of tile `t` (wave 0, lane w): misplaced keys of part
// [s0, s1) on side `side` in the words that precede w in rank order
// (ascending offsets on the left side, descending on the right side).
template <int NT>
__device__ __forceinline__ void ip_word_prefix(const Args& a, uint32_t t, int s0, int s1, int side, uint32_t* wpre) {
    static_assert(kIpWords == 64, "one class word per lane");
    const int tid = threadIdx.x;
    if (tid < 64) {
        const uint64_t word = a.ipmask[static_cast<size_t>(t) * kIpWords + tid];
        const uint64_t m = misplaced_bits(word, tid, s0, s1, side);
        const uint64_t c = static_cast<uint64_t>(__popcll(m));
        const uint64_t inc = wave_inclusive_sum(c, tid);
        const uint64_t tot = bcast64(inc, 63);
        wpre[tid] = static_cast<uint32_t>(side == 0 ? inc - c : tot - inc);
    }
}

// Rank (within its tile part, in rank order) of the key at lane `lane` of
// class word w, whose misplaced bits are m.
__device__ __forceinline__ uint32_t ip_local_rank(uint64_t m, uint32_t before, int lane, int side) {
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint64_t above = lane == 63 ? 0ull : (~0ull << (lane + 1));
    return before + static_cast<uint32_t>(__popcll(m & (side == 0 ? below : above)));
}

template <int DT, class V, int NT, int EPT>
__device__ void ip_exchange_tile(const Args& a, int p, uint32_t t, IpLds<DT, V, NT, EPT>& L) {
    using R = typename KeyT<DT>::raw;
    using VS = typename ValStore<V>::type;
    constexpr bool HV = !std::is_same<V, NoVal>::value;
    constexpr int T = NT * EPT;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const TileDesc td = a.tile_desc[t];
    const SegDesc& sd = a.segs[p][td.si];
    const int64_t b = td.lo + static_cast<int64_t>(sd.cursor & 0xffffffffull);
    const int aside = (sd.pad & kSegARight) ? 1 : 0, bside = 1 - aside;
    const uint32_t c = a.iptile[t].mis[aside];
    if (c == 0) return;
    const uint32_t tl = td.t0 + sd.nt - 1;  // the segment's last tile
    const uint32_t M = a.iptile[tl].rank[1];
    const uint32_t base = aside == 0 ? a.iptile[t].rank[0] : M - a.iptile[t].rank[1];
    const int64_t tlo = td.lo + static_cast<int64_t>(t - td.t0) * T;
    const int len = static_cast<int>(td.hi - tlo < T ? td.hi - tlo : T);
    int s0, s1;
    side_part(tlo, len, b, aside, s0, s1);
    R* keys = static_cast<R*>(a.x_keys);
    VS* vals = static_cast<VS*>(a.x_vals);
    const uint64_t* mw = a.ipmask + static_cast<size_t>(t) * kIpWords;

    // 1. the owning tile's part into LDS; the tile offset of each owned
    // misplaced key by its rank
    ip_word_prefix<NT>(a, t, s0, s1, aside, L.wpre);
    if (tid == 0) {
        // first partner tile: bside 0 (left, ascending ranks) the first tile
        // whose ranks reach past `base`; bside 1 (right, ranks from the
        // right end) the first tile whose running sum reaches M - base
        uint32_t lo_i = td.t0, hi_i = tl;
        while (lo_i < hi_i) {
            const uint32_t mid = (lo_i + hi_i) >> 1;
            const bool past = bside == 0 ? a.iptile[mid].rank[0] + a.iptile[mid].mis[0] > base
                                         : a.iptile[mid].rank[1] >= M - base;
            if (past) hi_i = mid; else lo_i = mid + 1;
        }
        L.u = lo_i;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int o = r * NT + tid;
        if (o >= s0 && o < s1) {
            L.k[o] = keys[tlo + o];
            if constexpr (HV) L.v[o] = vals[tlo + o];
        }
    }
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int w = r * NW + wv;
        const uint64_t m = misplaced_bits(mw[w], w, s0, s1, aside);
        if ((m >> lane) & 1ull) L.pos[ip_local_rank(m, L.wpre[w], lane, aside)] = static_cast<uint16_t>(r * NT + tid);
    }
    const uint32_t first = L.u;
    __syncthreads();

    // 2. partner tiles in rank order; each swaps its share of ranks
    // [base, base + c) with the owned keys through LDS
    uint32_t covered = 0;
    uint32_t u = first;
    while (covered < c) {
        if (u < td.t0 || u > tl) {
            if (tid == 0) atomicOr(&a.ctl->error, ERR_OVERFLOW);  // inconsistent running sums
            break;
        }
        const uint32_t umis = a.iptile[u].mis[bside];
        const uint32_t ubase = bside == 0 ? a.iptile[u].rank[0] : M - a.iptile[u].rank[1];
        const uint32_t r0 = ubase > base ? ubase : base;
        const uint32_t r1 = ubase + umis < base + c ? ubase + umis : base + c;
        if (r1 > r0) {
            const int64_t ulo = td.lo + static_cast<int64_t>(u - td.t0) * T;
            const int ulen = static_cast<int>(td.hi - ulo < T ? td.hi - ulo : T);
            int q0, q1;
            side_part(ulo, ulen, b, bside, q0, q1);
            const uint64_t* uw = a.ipmask + static_cast<size_t>(u) * kIpWords;
            ip_word_prefix<NT>(a, u, q0, q1, bside, L.wpre);
            if (tid == 0) {
                L.omin = 0xffffffffu;
                L.omax = 0u;
            }
            __syncthreads();
            // which of this thread's keys are partners, and their ranks
            uint32_t idx[EPT];
            uint32_t mine = 0;
            uint32_t omin = 0xffffffffu, omax = 0;
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                const int w = r * NW + wv;
                const uint64_t m = misplaced_bits(uw[w], w, q0, q1, bside);
                const uint32_t rk = ubase + ip_local_rank(m, L.wpre[w], lane, bside);
                const bool hit = ((m >> lane) & 1ull) && rk >= r0 && rk < r1;
                idx[r] = rk - base;
                if (hit) {
                    mine |= 1u << r;
                    const uint32_t o = static_cast<uint32_t>(r * NT + tid);
                    omin = o < omin ? o : omin;
                    omax = o > omax ? o : omax;
                }
            }
            if (mine) {
                atomicMin(&L.omin, omin);
                atomicMax(&L.omax, omax);
            }
            __syncthreads();
            const uint32_t lo_o = L.omin, hi_o = L.omax;
            // the owned range [lo_o, hi_o] of the partner tile: read, swap,
            // write back
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                const uint32_t o = static_cast<uint32_t>(r * NT + tid);
                if (o >= lo_o && o <= hi_o) {
                    R x = keys[ulo + o];
                    VS y{};
                    if constexpr (HV) y = vals[ulo + o];
                    if ((mine >> r) & 1u) {
                        const int op = L.pos[idx[r]];
                        const R x_own = L.k[op];
                        L.k[op] = x;
                        x = x_own;
                        if constexpr (HV) {
                            const VS y_own = L.v[op];
                            L.v[op] = y;
                            y = y_own;
                        }
                    }
                    keys[ulo + o] = x;
                    if constexpr (HV) vals[ulo + o] = y;
                }
            }
            covered += r1 - r0;
            __syncthreads();  // wpre, omin and omax are free again
        }
        u = bside == 0 ? u + 1 : u - 1;
    }
    __syncthreads();
    // 3. the owning tile's part back in place
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int o = r * NT + tid;
        if (o >= s0 && o < s1) {
            keys[tlo + o] = L.k[o];
            if constexpr (HV) vals[tlo + o] = L.v[o];
        }
    }
    __syncthreads();  // LDS is free for the next tile
}

template <int DT, class V, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_ip_exchange(Args a) {
    __shared__ IpLds<DT, V, NT, EPT> s_lds;
    const Ctl* c = a.ctl;
    const int p = a.level & 1;
    uint32_t ntiles = static_cast<uint32_t>(c->lc[p].segs >> 32);
    if (ntiles > a.cap_tile) ntiles = a.cap_tile;
    if (blockIdx.x >= ntiles || c->error) return;  // (an error latched by an earlier step: nothing runs)
    ip_exchange_tile<DT, V, NT, EPT>(a, p, blockIdx.x, s_lds);
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
        uint32_t depth = 0;
        uint64_t pv = 0, praw = 0;
        if (valid) {
            const SegDesc sd = a.segs[p][si];
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
            } else {
                clo[0] = sd.lo;
                chi[0] = b;
                const int64_t right = sd.hi - b;
                if (right > ne) {  // not all equal to the pivot
                    clo[1] = b;
                    chi[1] = sd.hi;
                    forced[1] = ne > 0 && (nl == 0 || 8 * ne >= right);
                }
            }
        }
        int kind[2], cls[2];
        uint32_t nt[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t m = chi[h] - clo[h];
            kind[h] = m <= 1 ? 0 : (m > S ? 1 : 2);
            nt[h] = kind[h] == 1 ? seg_tiles(clo[h], chi[h], T) : 0u;
            cls[h] = kind[h] == 2 ? small_class(m) : -1;
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
                else dst[idx] = SmallItem{clo[h], chi[h]};
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
    __shared__ uint32_t s_w[2 * (NT / 64)];
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
        for (uint32_t t = 0; t < ntile; ++t) ip_count_tile<DT, NT, EPT>(a, p, t, s_w);
        tail_sync();
        for (uint32_t si = 0; si < nseg; ++si) ip_scan_segment<NT>(a, p, si, s_w);
        tail_sync();
        if (tail_error(c)) break;
        auto& xl = *reinterpret_cast<IpLds<DT, V, NT, EPT>*>(s_raw);
        for (uint32_t t = 0; t < ntile; ++t) ip_exchange_tile<DT, V, NT, EPT>(a, p, t, xl);
        tail_sync();
        ip_complete_body(a, L, 0, 1);
        tail_sync();
    }
}

}  // namespace bqs
