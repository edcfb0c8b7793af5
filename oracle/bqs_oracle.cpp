// BlockQuicksort oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded CPU implementation of BlockQuicksort as
// Edelkamp & Weiss define it ("BlockQuicksort: How Branch Mispredictions
// don't affect Quicksort", arXiv 1604.06697).  It exists to check the GPU
// library: only the test suite, the smoke check and the benchmark's CPU
// baseline load it.  It shares no code, header, table or helper with the
// GPU path and never calls into it.
//
// What it follows, section by section of the paper:
//   * problem statement: sort a sequence of a totally ordered universe
//     ascending, in place (Introduction);
//   * Quicksort main loop: explicit stack (Sedgewick), pivot excluded from
//     the recursion, Introsort depth limit 2*log n + 3 then Heapsort,
//     Insertionsort for sub-arrays of at most 16 elements, median-of-three
//     pivot (Section 2, "Quicksort and improvements"; Algorithm 1);
//   * block partitioning: scanning phase that stores offsets of misplaced
//     elements into two buffers offsets_L / offsets_R with a counter that is
//     increased by the Boolean comparison outcome, rearrangement phase that
//     swaps min(num_L, num_R) pairs, block cursors advancing by B, and the
//     final one-or-two short blocks followed by a Lomuto-like move of what is
//     left in one buffer (Section 3, Algorithm 3 and the prose after it);
//   * B = 128 (Section 3.1) and the insertion-sort threshold 16 (Section 2).
//
// Readings where the paper is silent or inconsistent (each one is listed in
// the design notes):
//   * Algorithm 3 prints the scan predicates as (pivot >= A) for the left and
//     (pivot <= A) for the right buffer; the prose says offsets_L collects
//     elements greater or equal the pivot.  The prose (and Hoare's rule) is
//     followed: left buffer <- A >= pivot, right buffer <- A <= pivot.
//   * The third median-of-three sample is the last element of the range.
//   * Insertionsort and Heapsort are not given; textbook versions are used
//     (straight insertion, Knuth 5.2.1; Williams/Floyd heapsort).
//   * Floating-point keys use the IEEE-754 total order restricted to
//     non-NaN values: -0.0 < +0.0.  A NaN input is rejected.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -shared -fPIC -o liboracle.so bqs_oracle.cpp
// (no fused multiply-add: the Vector comparator rounds every product and sum)
// A planted mistake for the pin tests is selected with -DORACLE_MUTANT=k.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

extern "C" {

// Tuning knobs and counters.  Zero-initialised fields select the paper's
// defaults.
typedef struct {
    int64_t block;          // B; 0 selects 128
    int64_t is_thresh;      // insertion-sort threshold; 0 selects 16
    int64_t depth_limit;    // < 0 selects 2*floor(log2 n) + 3
    int32_t check;          // != 0: verify each partition's postcondition
    int32_t reserved;
    // outputs (accumulated)
    int64_t comparisons;
    int64_t partitions;
    int64_t heapsorts;
    int64_t check_failures;
} oracle_params;

enum { OR_I32 = 1, OR_U32 = 2, OR_I64 = 3, OR_U64 = 4, OR_F32 = 5, OR_F64 = 6 };
enum { OR_OK = 0, OR_EINVAL = 1, OR_EDTYPE = 2, OR_ENAN = 5 };

}  // extern "C"

namespace {

struct NoVal {};

template <class K, class V>
struct Rec {
    K key;
    V val;
};

template <class K>
struct Rec<K, NoVal> {
    K key;
};

// Strict weak order on keys.  Integers: the usual <.  Floating point: <,
// with -0.0 ordered before +0.0 (IEEE-754 totalOrder on non-NaN values).
template <class K, bool kFloat = std::is_floating_point<K>::value>
struct KeyLess {
    static bool lt(K a, K b) { return a < b; }
};

template <class K>
struct KeyLess<K, true> {
    static bool lt(K a, K b) {
#if ORACLE_MUTANT == 8
        return a < b;  // planted: ignores the order of the two zeros
#else
        return a < b || (a == b && std::signbit(a) && !std::signbit(b));
#endif
    }
};

// The paper's two large element types (Section 4, experimental setup):
// Vector, ten doubles ordered by the sum of the squares of the components,
// computed afresh at every comparison (left to right: x0*x0 + x1*x1 + ...);
// Record, 21 int32 of which only the first is compared.
struct VectorRec {
    double x[10];
};
struct RecordRec {
    int32_t x[21];
};

inline double sum_of_squares(const VectorRec& v) {
    double s = v.x[0] * v.x[0];
    for (int i = 1; i < 10; ++i) s = s + v.x[i] * v.x[i];
    return s;
}

template <class R>
inline bool rec_less(const R& a, const R& b) {
    return KeyLess<decltype(a.key)>::lt(a.key, b.key);
}
inline bool rec_less(const VectorRec& a, const VectorRec& b) { return sum_of_squares(a) < sum_of_squares(b); }
inline bool rec_less(const RecordRec& a, const RecordRec& b) { return a.x[0] < b.x[0]; }

template <class R>
struct Less {
    int64_t* count;
    bool operator()(const R& a, const R& b) const {
        ++*count;
        return rec_less(a, b);
    }
};

template <class R>
inline void swap_rec(R* A, int64_t i, int64_t j) {
    R t = A[i];
    A[i] = A[j];
    A[j] = t;
}

// ---------------------------------------------------------------------------
// Base cases (Section 2): Insertionsort for small sub-arrays, Heapsort when
// the recursion depth limit is exceeded.

template <class R, class L>
void insertion_sort(R* A, int64_t lo, int64_t hi, L& less) {
    // Straight insertion: grow a sorted prefix A[lo..i) one element at a time.
    for (int64_t i = lo + 1; i < hi; ++i) {
        R x = A[i];
        int64_t j = i;
#if ORACLE_MUTANT == 6
        while (j > lo + 1 && less(x, A[j - 1])) {  // planted: never reaches lo
#else
        while (j > lo && less(x, A[j - 1])) {
#endif
            A[j] = A[j - 1];
            --j;
        }
        A[j] = x;
    }
}

template <class R, class L>
void sift_down(R* H, int64_t root, int64_t size, L& less) {
    // H is a 0-based max-heap view; children of k are 2k+1 and 2k+2.
    for (;;) {
#if ORACLE_MUTANT == 7
        int64_t child = 2 * root + 2;  // planted: skips the left child
#else
        int64_t child = 2 * root + 1;
#endif
        if (child >= size) return;
        if (child + 1 < size && less(H[child], H[child + 1])) ++child;
        if (!less(H[root], H[child])) return;
        swap_rec(H, root, child);
        root = child;
    }
}

template <class R, class L>
void heap_sort(R* A, int64_t lo, int64_t hi, L& less) {
    R* H = A + lo;
    int64_t n = hi - lo;
    for (int64_t k = n / 2 - 1; k >= 0; --k) sift_down(H, k, n, less);
    for (int64_t end = n - 1; end > 0; --end) {
        swap_rec(H, 0, end);
        sift_down(H, 0, end, less);
    }
}

// ---------------------------------------------------------------------------
// Block partitioning (Section 3, Algorithm 3).
//
// A buffer holds offsets of scanned elements that lie on the wrong side of
// the pivot.  `start` is the first offset not yet used by a swap, `num` the
// number of offsets still waiting.

struct Buffer {
    std::vector<int64_t> offsets;
    int64_t start = 0;
    int64_t num = 0;
    explicit Buffer(int64_t B) : offsets(static_cast<size_t>(B > 0 ? B : 1)) {}
};

// Scanning phase, left side: looks at A[l], A[l+1], ..., A[l+len-1].  The
// offset is always written; the counter only advances when the element is
// >= pivot, i.e. the comparison outcome is added as an integer.
template <class R, class L>
void scan_left(Buffer& bl, const R* A, int64_t l, int64_t len, const R& pivot, L& less) {
    bl.start = 0;
    bl.num = 0;
    for (int64_t i = 0; i < len; ++i) {
        bl.offsets[bl.num] = i;
#if ORACLE_MUTANT == 1
        bl.num += static_cast<int64_t>(less(A[l + i], pivot));  // planted: wrong direction
#else
        bl.num += static_cast<int64_t>(!less(A[l + i], pivot));
#endif
    }
}

// Scanning phase, right side: looks at A[r], A[r-1], ..., A[r-len+1] and
// records the offsets (counted from r downwards) of elements <= pivot.
template <class R, class L>
void scan_right(Buffer& br, const R* A, int64_t r, int64_t len, const R& pivot, L& less) {
    br.start = 0;
    br.num = 0;
    for (int64_t i = 0; i < len; ++i) {
        br.offsets[br.num] = i;
        br.num += static_cast<int64_t>(!less(pivot, A[r - i]));
    }
}

// Rearrangement phase: swap as many misplaced pairs as both buffers hold.
template <class R>
void rearrange(R* A, int64_t l, int64_t r, Buffer& bl, Buffer& br) {
    const int64_t num = bl.num < br.num ? bl.num : br.num;
    for (int64_t j = 0; j < num; ++j)
        swap_rec(A, l + bl.offsets[bl.start + j], r - br.offsets[br.start + j]);
    bl.num -= num;
    br.num -= num;
    bl.start += num;
    br.start += num;
}

// Partitions A[l..r] (inclusive; the pivot itself is parked outside, to the
// right of r) and returns `cut`: every element of A[l..cut) is <= pivot and
// every element of A[cut..r] is >= pivot.
template <class R, class L>
int64_t block_partition(R* A, int64_t l, int64_t r, const R& pivot, int64_t B, L& less) {
    Buffer bl(B), br(B);

    // Main loop: while more than two blocks remain, refill whichever buffer
    // ran empty, swap, and advance the cursor of every emptied side by B.
    while (r - l + 1 > 2 * B) {
        if (bl.num == 0) scan_left(bl, A, l, B, pivot, less);
        if (br.num == 0) scan_right(br, A, r, B, pivot, less);
        rearrange(A, l, r, bl, br);
        if (bl.num == 0) l += B;
        if (br.num == 0) r -= B;
    }

    // Final iteration: the at most 2B remaining elements are scanned as one
    // or two shorter blocks.  A side whose buffer still holds offsets keeps
    // its full block of B; the other side gets what lies in between.
    const int64_t width = r - l + 1;
    int64_t lenL, lenR;
    if (bl.num == 0 && br.num == 0) {
        lenL = width / 2;
#if ORACLE_MUTANT == 2
        lenR = width - lenL - 1;  // planted: forgets one element
#else
        lenR = width - lenL;
#endif
        scan_left(bl, A, l, lenL, pivot, less);
        scan_right(br, A, r, lenR, pivot, less);
    } else if (bl.num == 0) {
        lenR = B;
        lenL = width - B;
        scan_left(bl, A, l, lenL, pivot, less);
    } else {
        lenL = B;
        lenR = width - B;
        scan_right(br, A, r, lenR, pivot, less);
    }
    rearrange(A, l, r, bl, br);
    if (bl.num == 0) l += lenL;
    if (br.num == 0) r -= lenR;

    // At most one buffer is non-empty now and [l, r] is exactly its block.
    // Move the elements it still points to to the far end of the block, in
    // one pass over the buffer (Lomuto-like, without comparisons).
    if (bl.num > 0) {
        int64_t upper = r - l;  // offset of the rightmost free slot
        for (int64_t q = bl.start + bl.num - 1; q >= bl.start; --q) {
            swap_rec(A, l + bl.offsets[q], l + upper);
            --upper;
        }
#if ORACLE_MUTANT == 4
        return l + upper;  // planted: off by one
#else
        return l + upper + 1;
#endif
    }
    if (br.num > 0) {
        int64_t upper = r - l;  // offset (from r) of the leftmost free slot
        for (int64_t q = br.start + br.num - 1; q >= br.start; --q) {
            swap_rec(A, r - br.offsets[q], r - upper);
            --upper;
        }
#if ORACLE_MUTANT == 5
        return r - upper + 1;  // planted: off by one
#else
        return r - upper;
#endif
    }
    return l;
}

// One partitioning step on A[lo, hi) with hi - lo >= 3: median-of-three
// pivot, block partition of the inner range, pivot moved to its final slot.
template <class R, class L>
int64_t partition(R* A, int64_t lo, int64_t hi, int64_t B, L& less) {
    const int64_t mid = lo + (hi - lo) / 2;
    auto cmpx = [&](int64_t i, int64_t j) {
        if (less(A[j], A[i])) swap_rec(A, i, j);
    };
    cmpx(lo, mid);
    cmpx(mid, hi - 1);
#if ORACLE_MUTANT != 3
    cmpx(lo, mid);
#endif
    // Now A[lo] <= A[mid] <= A[hi-1]: the two outer samples already lie on
    // their sides.  Park the pivot next to the right sample.
    const int64_t park = hi - 2;
    swap_rec(A, mid, park);
    const R pivot = A[park];
    const int64_t cut = block_partition(A, lo + 1, park - 1, pivot, B, less);
    swap_rec(A, cut, park);
    return cut;
}

template <class R, class L>
bool partition_ok(const R* A, int64_t lo, int64_t hi, int64_t cut, L& less) {
    for (int64_t i = lo; i < cut; ++i)
        if (less(A[cut], A[i])) return false;
    for (int64_t i = cut + 1; i < hi; ++i)
        if (less(A[i], A[cut])) return false;
    return true;
}

int64_t floor_log2(int64_t n) {
    int64_t k = 0;
    while (n > 1) {
        n >>= 1;
        ++k;
    }
    return k;
}

// Quicksort main loop (Algorithm 1 with the improvements of Section 2).
template <class R>
void block_quicksort(R* A, int64_t n, oracle_params* p) {
    if (n <= 1) return;
    const int64_t B = p->block > 0 ? p->block : 128;
    const int64_t IS = p->is_thresh > 0 ? p->is_thresh : 16;
    const int64_t limit = p->depth_limit >= 0 ? p->depth_limit : 2 * floor_log2(n) + 3;
    Less<R> less{&p->comparisons};
    int64_t scratch = 0;
    Less<R> uncounted{&scratch};

    struct Item {
        int64_t lo, hi, depth;
    };
    std::vector<Item> stack;
    Item cur{0, n, 0};
    for (;;) {
        const int64_t size = cur.hi - cur.lo;
        if (cur.depth < limit && size > IS && size >= 3) {
            const int64_t cut = partition(A, cur.lo, cur.hi, B, less);
            ++p->partitions;
            if (p->check && !partition_ok(A, cur.lo, cur.hi, cut, uncounted)) ++p->check_failures;
            // Sedgewick: keep the smaller side, push the larger one.  The
            // pivot is in its final place and takes part in neither.
            const Item left{cur.lo, cut, cur.depth + 1};
            const Item right{cut + 1, cur.hi, cur.depth + 1};
            if (cut - cur.lo > cur.hi - cut) {
                stack.push_back(left);
                cur = right;
            } else {
                stack.push_back(right);
                cur = left;
            }
        } else {
            if (size > IS) {
                heap_sort(A, cur.lo, cur.hi, less);
                ++p->heapsorts;
            } else {
                insertion_sort(A, cur.lo, cur.hi, less);
            }
            if (stack.empty()) break;
            cur = stack.back();
            stack.pop_back();
        }
    }
}

template <class K>
bool has_nan(const K* keys, int64_t n) {
    if (!std::is_floating_point<K>::value) return false;
    for (int64_t i = 0; i < n; ++i)
        if (keys[i] != keys[i]) return true;
    return false;
}

template <class K>
int sort_keys(void* keys, int64_t n, oracle_params* p) {
    using R = Rec<K, NoVal>;
    static_assert(sizeof(R) == sizeof(K), "record must be the bare key");
    if (has_nan(static_cast<K*>(keys), n)) return OR_ENAN;
    block_quicksort(static_cast<R*>(keys), n, p);
    return OR_OK;
}

template <class K, class V>
int sort_pairs_t(void* keys, void* vals, int64_t n, oracle_params* p) {
    using R = Rec<K, V>;
    K* k = static_cast<K*>(keys);
    V* v = static_cast<V*>(vals);
    if (has_nan(k, n)) return OR_ENAN;
    std::vector<R> recs(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) recs[i] = R{k[i], v[i]};
    block_quicksort(recs.data(), n, p);
    for (int64_t i = 0; i < n; ++i) {
        k[i] = recs[i].key;
        v[i] = recs[i].val;
    }
    return OR_OK;
}

template <class K>
int64_t partition_once_t(void* keys, int64_t lo, int64_t hi, oracle_params* p) {
    using R = Rec<K, NoVal>;
    R* A = static_cast<R*>(keys);
    Less<R> less{&p->comparisons};
    const int64_t B = p->block > 0 ? p->block : 128;
    return partition(A, lo, hi, B, less);
}

size_t key_bytes(int dtype) {
    switch (dtype) {
        case OR_I32: case OR_U32: case OR_F32: return 4;
        case OR_I64: case OR_U64: case OR_F64: return 8;
        default: return 0;
    }
}

int dispatch_keys(void* keys, int64_t n, int dtype, oracle_params* p) {
    switch (dtype) {
        case OR_I32: return sort_keys<int32_t>(keys, n, p);
        case OR_U32: return sort_keys<uint32_t>(keys, n, p);
        case OR_I64: return sort_keys<int64_t>(keys, n, p);
        case OR_U64: return sort_keys<uint64_t>(keys, n, p);
        case OR_F32: return sort_keys<float>(keys, n, p);
        case OR_F64: return sort_keys<double>(keys, n, p);
        default: return OR_EDTYPE;
    }
}

template <class V>
int dispatch_pairs(void* keys, void* vals, int64_t n, int dtype, oracle_params* p) {
    switch (dtype) {
        case OR_I32: return sort_pairs_t<int32_t, V>(keys, vals, n, p);
        case OR_U32: return sort_pairs_t<uint32_t, V>(keys, vals, n, p);
        case OR_I64: return sort_pairs_t<int64_t, V>(keys, vals, n, p);
        case OR_U64: return sort_pairs_t<uint64_t, V>(keys, vals, n, p);
        case OR_F32: return sort_pairs_t<float, V>(keys, vals, n, p);
        case OR_F64: return sort_pairs_t<double, V>(keys, vals, n, p);
        default: return OR_EDTYPE;
    }
}

}  // namespace

extern "C" {

// Sorts keys[0..n) ascending in place.  Returns OR_OK, OR_EINVAL (bad
// pointer or n), OR_EDTYPE or OR_ENAN.
int oracle_sort(void* keys, int64_t n, int dtype, oracle_params* p) {
    if (n < 0 || (n > 0 && !keys) || !p) return OR_EINVAL;
    return dispatch_keys(keys, n, dtype, p);
}

// Sorts (keys, vals) records by key; vals are 4- or 8-byte payloads that
// travel with their key.  Unstable, like the paper's algorithm.
int oracle_sort_pairs(void* keys, void* vals, int64_t n, int dtype, int val_bytes, oracle_params* p) {
    if (n < 0 || (n > 0 && (!keys || !vals)) || !p) return OR_EINVAL;
    if (val_bytes == 4) return dispatch_pairs<uint32_t>(keys, vals, n, dtype, p);
    if (val_bytes == 8) return dispatch_pairs<uint64_t>(keys, vals, n, dtype, p);
    return OR_EDTYPE;
}

// Sorts each segment keys[offsets[i] .. offsets[i+1]) independently.
int oracle_sort_segments(void* keys, const int64_t* offsets, int64_t k, int dtype, oracle_params* p) {
    if (k < 0 || !p || (k > 0 && !offsets)) return OR_EINVAL;
    const size_t kb = key_bytes(dtype);
    if (!kb) return OR_EDTYPE;
    for (int64_t i = 0; i < k; ++i)
        if (offsets[i + 1] < offsets[i] || offsets[i] < 0) return OR_EINVAL;
    for (int64_t i = 0; i < k; ++i) {
        char* base = static_cast<char*>(keys) + static_cast<size_t>(offsets[i]) * kb;
        const int rc = dispatch_keys(base, offsets[i + 1] - offsets[i], dtype, p);
        if (rc != OR_OK) return rc;
    }
    return OR_OK;
}

// One median-of-three + block-partition step on keys[lo, hi) (test hook).
// Returns the pivot's final index, or -1 on bad arguments.
int64_t oracle_partition(void* keys, int64_t lo, int64_t hi, int dtype, oracle_params* p) {
    if (!keys || !p || lo < 0 || hi - lo < 3) return -1;
    switch (dtype) {
        case OR_I32: return partition_once_t<int32_t>(keys, lo, hi, p);
        case OR_U32: return partition_once_t<uint32_t>(keys, lo, hi, p);
        case OR_I64: return partition_once_t<int64_t>(keys, lo, hi, p);
        case OR_U64: return partition_once_t<uint64_t>(keys, lo, hi, p);
        case OR_F32: return partition_once_t<float>(keys, lo, hi, p);
        case OR_F64: return partition_once_t<double>(keys, lo, hi, p);
        default: return -1;
    }
}

// Sorts n records of the paper's Vector (kind 1, 80 bytes) or Record (kind
// 2, 84 bytes) type in place with their comparators.
int oracle_sort_records(void* recs, int64_t n, int kind, oracle_params* p) {
    if (n < 0 || (n > 0 && !recs) || !p) return OR_EINVAL;
    if (kind == 1) {
        block_quicksort(static_cast<VectorRec*>(recs), n, p);
        return OR_OK;
    }
    if (kind == 2) {
        block_quicksort(static_cast<RecordRec*>(recs), n, p);
        return OR_OK;
    }
    return OR_EDTYPE;
}

// The host's std::sort with the oracle's key order (the paper's comparison
// baseline, Section 4), called as a library routine: the CPU context timed
// beside the oracle.  Returns OR_OK, OR_EINVAL, OR_EDTYPE or OR_ENAN.
int oracle_std_sort(void* keys, int64_t n, int dtype) {
    if (n < 0 || (n > 0 && !keys)) return OR_EINVAL;
    switch (dtype) {
        case OR_I32: std::sort(static_cast<int32_t*>(keys), static_cast<int32_t*>(keys) + n); return OR_OK;
        case OR_U32: std::sort(static_cast<uint32_t*>(keys), static_cast<uint32_t*>(keys) + n); return OR_OK;
        case OR_I64: std::sort(static_cast<int64_t*>(keys), static_cast<int64_t*>(keys) + n); return OR_OK;
        case OR_U64: std::sort(static_cast<uint64_t*>(keys), static_cast<uint64_t*>(keys) + n); return OR_OK;
        case OR_F32:
            if (has_nan(static_cast<float*>(keys), n)) return OR_ENAN;
            std::sort(static_cast<float*>(keys), static_cast<float*>(keys) + n, KeyLess<float>::lt);
            return OR_OK;
        case OR_F64:
            if (has_nan(static_cast<double*>(keys), n)) return OR_ENAN;
            std::sort(static_cast<double*>(keys), static_cast<double*>(keys) + n, KeyLess<double>::lt);
            return OR_OK;
        default: return OR_EDTYPE;
    }
}

int oracle_mutant(void) { return ORACLE_MUTANT; }

}  // extern "C"
