// gfx950 kernels for sort-based grouping with early aggregation and wide
// merging (Do, Graefe, Naughton).
//
// The device path has four kinds of work:
//  * partitioning (sample, histogram, scatter): an unsorted batch is split
//    into key ranges by splitters chosen from a sample -- the upper level of
//    the ordered in-memory index (Section 3.3: an ordered index; interpolation
//    or batched search locates a key's range);
//  * leaf sort-reduce: one workgroup sorts a key range in LDS and collapses
//    equal adjacent keys into state rows (Section 6.1: sort the batch within
//    the cache to detect duplicates; Section 2.1: in-stream grouping over
//    sorted data);
//  * merge with aggregation: two sorted runs of unique keys are merged and
//    equal keys combined (Section 3: absorbing a batch into the index;
//    Section 4: merging runs with aggregation);
//  * scans and copies that place variable-length outputs.
//
// All kernels are written for wave64 (CDNA) and use only vector memory
// instructions for global stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "isa_internal.h"

namespace isa {

// ---------------------------------------------------------------------------
// Row helpers
// ---------------------------------------------------------------------------

struct Agg {
    uint64_t key;
    uint64_t cnt;
    uint64_t sum;  // int64 sum carried as uint64 so that it wraps
    int64_t mn, mx;
    double fs;
};

__device__ __forceinline__ Agg load_agg(const ColView& v, uint64_t i) {
    Agg a;
    const uint64_t o = i * v.stride;
    a.key = v.key[o];
    a.cnt = v.cnt ? v.cnt[o] : 1ull;
    a.sum = v.sum ? (uint64_t)v.sum[o] : 0ull;
    a.mn = v.mn ? v.mn[o] : INT64_MAX;
    a.mx = v.mx ? v.mx[o] : INT64_MIN;
    a.fs = v.fs ? v.fs[o] : 0.0;
    return a;
}

__device__ __forceinline__ void load_payload(const ColView& v, uint64_t i, Agg& a) {
    const uint64_t o = i * v.stride;
    a.cnt = v.cnt ? v.cnt[o] : 1ull;
    a.sum = v.sum ? (uint64_t)v.sum[o] : 0ull;
    a.mn = v.mn ? v.mn[o] : INT64_MAX;
    a.mx = v.mx ? v.mx[o] : INT64_MIN;
    a.fs = v.fs ? v.fs[o] : 0.0;
}

__device__ __forceinline__ void combine(Agg& a, const Agg& b) {
    a.cnt += b.cnt;
    a.sum += b.sum;
    a.mn = b.mn < a.mn ? b.mn : a.mn;
    a.mx = b.mx > a.mx ? b.mx : a.mx;
    a.fs += b.fs;
}

__device__ __forceinline__ void empty_agg(Agg& a) {
    a.cnt = 0;
    a.sum = 0;
    a.mn = INT64_MAX;
    a.mx = INT64_MIN;
    a.fs = 0.0;
}

__device__ __forceinline__ void store_agg(const OutView& o, uint64_t i, const Agg& a) {
    const uint64_t p = i * o.stride;
    o.key[p] = a.key;
    if (o.cnt) o.cnt[p] = a.cnt;
    if (o.sum) o.sum[p] = (int64_t)a.sum;
    if (o.mn) o.mn[p] = a.mn;
    if (o.mx) o.mx[p] = a.mx;
    if (o.fs) o.fs[p] = a.fs;
}

// Write one row into a row-major partition buffer.
__device__ __forceinline__ void store_row(uint64_t* row, const Layout& L, const Agg& a) {
    row[0] = a.key;
    if (L.cnt >= 0) row[L.cnt] = a.cnt;
    if (L.sum >= 0) row[L.sum] = a.sum;
    if (L.mn >= 0 && L.mn != L.sum) row[L.mn] = (uint64_t)a.mn;
    if (L.mx >= 0 && L.mx != L.sum) row[L.mx] = (uint64_t)a.mx;
    if (L.fs >= 0) row[L.fs] = __double_as_longlong(a.fs);
}

__device__ __forceinline__ int bit_length(uint64_t x) { return x ? 64 - __clzll(x) : 0; }

// ---------------------------------------------------------------------------
// Wave and block scans
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan over the NT threads of the block; s_tmp holds NT/64+1 words.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_tmp, uint32_t& total) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_scan(x);
    if (lane == 63) s_tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < NW; ++i) {
            uint32_t c = s_tmp[i];
            s_tmp[i] = run;
            run += c;
        }
        s_tmp[NW] = run;
    }
    __syncthreads();
    uint32_t r = s_tmp[w] + inc - x;
    total = s_tmp[NW];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Wave-level rank by digit: lanes with equal digit find each other through
// one ballot per digit bit; rank = earlier lanes with the same digit plus the
// wave's running count of that digit (kept in LDS).  Stable in lane order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t wave_match(uint32_t d, int dbits, uint64_t active) {
    uint64_t match = active;
    for (int b = 0; b < dbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        match &= bit ? bal : ~bal;
    }
    return match;
}

// ---------------------------------------------------------------------------
// Block radix sort of NT*IPT (key, val) pairs held in registers in
// warp-striped order (item j of lane l in wave w is logical item
// w*64*IPT + j*64 + l).  Sorts on bits [0, nbits) of the keys, stably, eight
// bits per pass.  Leaves the sorted pairs in s_key/s_val at position pad(p).
// ---------------------------------------------------------------------------

template <int NT, int IPT>
struct SortSmem {
    static constexpr int N = NT * IPT;
    static constexpr int NP = N + N / 16;  // padded for conflict-light blocked reads
    uint64_t key[NP];
    uint32_t val[NP];
    uint32_t cnt[(NT / 64) * 256];
    uint32_t dbase[256];
    uint32_t tmp[NT / 64 + 1];
};

__device__ __forceinline__ int pad16(int p) { return p + (p >> 4); }

template <int NT, int IPT>
__device__ void block_radix_sort(uint64_t (&k)[IPT], uint32_t (&v)[IPT], int nbits,
                                 SortSmem<NT, IPT>& s) {
    static_assert(NT >= 256, "digit scan uses 256 threads");
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    if (nbits <= 0) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int p = w * 64 * IPT + j * 64 + lane;
            s.key[pad16(p)] = k[j];
            s.val[pad16(p)] = v[j];
        }
        __syncthreads();
        return;
    }
    for (int shift = 0; shift < nbits; shift += 8) {
        const int dbits = (nbits - shift) < 8 ? (nbits - shift) : 8;
        const uint32_t dmask = (1u << dbits) - 1u;
        const bool last = shift + 8 >= nbits;
        uint32_t* wc = s.cnt + w * 256;
        for (int i = lane; i < 256; i += 64) wc[i] = 0;
        uint32_t rank[IPT];
        uint32_t dig[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t d = (uint32_t)(k[j] >> shift) & dmask;
            const uint64_t match = wave_match(d, dbits, ~0ull);
            const uint32_t before = __popcll(match & lt);
            const uint32_t base = wc[d];
            if (before == 0) wc[d] = base + (uint32_t)__popcll(match);
            rank[j] = base + before;
            dig[j] = d;
        }
        __syncthreads();
        uint32_t run = 0;
        if (tid < 256) {
            for (int ww = 0; ww < NT / 64; ++ww) {
                const uint32_t c = s.cnt[ww * 256 + tid];
                s.cnt[ww * 256 + tid] = run;
                run += c;
            }
        }
        uint32_t total;
        const uint32_t excl = block_exclusive_scan<NT>(tid < 256 ? run : 0u, s.tmp, total);
        if (tid < 256) s.dbase[tid] = excl;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int pos = (int)(s.dbase[dig[j]] + s.cnt[w * 256 + dig[j]] + rank[j]);
            const int q = last ? pad16(pos) : pos;
            s.key[q] = k[j];
            s.val[q] = v[j];
        }
        __syncthreads();
        if (!last) {
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
                const int p = w * 64 * IPT + j * 64 + lane;
                k[j] = s.key[p];
                v[j] = s.val[p];
            }
            __syncthreads();
        }
    }
}

// Block-wide min and max of uint64 values.
template <int NT>
__device__ void block_minmax(uint64_t& mn, uint64_t& mx, uint64_t* s_tmp /* 2*NT/64 */) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t a = __shfl_xor(mn, off, 64);
        const uint64_t b = __shfl_xor(mx, off, 64);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if (lane == 0) {
        s_tmp[w] = mn;
        s_tmp[NW + w] = mx;
    }
    __syncthreads();
    mn = s_tmp[0];
    mx = s_tmp[NW];
    for (int i = 1; i < NW; ++i) {
        mn = s_tmp[i] < mn ? s_tmp[i] : mn;
        mx = s_tmp[NW + i] > mx ? s_tmp[NW + i] : mx;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Splitter selection: one workgroup per region sorts a stratified sample of
// SAMPLE_N keys and takes nb-1 quantiles as splitters.  A key that fills
// several quantiles is heavy; the next splitter is raised to key+1 so the heavy
// key gets a bucket of its own.  Splitters are padded to MAX_BUCKETS-1 with
// UINT64_MAX.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(LEAF_NT) k_sample(const Region* __restrict__ regions,
                                                    uint64_t* __restrict__ splitters) {
    constexpr int NT = LEAF_NT, IPT = LEAF_IPT;
    __shared__ SortSmem<NT, IPT> s;
    __shared__ uint64_t s_mm[2 * NT / 64];
    const Region R = regions[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t S = R.n < (uint64_t)SAMPLE_N ? R.n : (uint64_t)SAMPLE_N;
    uint64_t k[IPT];
    uint32_t v[IPT];
    uint64_t mn = ~0ull, mx = 0ull;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint64_t q = (uint64_t)(w * 64 * IPT + j * 64 + lane);
        v[j] = (uint32_t)q;
        if (q < S) {
            const uint64_t pos = (uint64_t)(((unsigned __int128)(2 * q + 1) * R.n) / (2 * S));
            k[j] = R.src.key[pos * R.src.stride];
            mn = k[j] < mn ? k[j] : mn;
            mx = k[j] > mx ? k[j] : mx;
        } else {
            k[j] = 0;
        }
    }
    block_minmax<NT>(mn, mx, s_mm);
    const uint64_t range = mx - mn;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint64_t q = (uint64_t)(w * 64 * IPT + j * 64 + lane);
        k[j] = q < S ? k[j] - mn : range;  // padding sorts last
    }
    block_radix_sort<NT, IPT>(k, v, bit_length(range), s);
    __shared__ uint64_t s_spl[MAX_BUCKETS];
    const uint32_t nb = R.nb;
    if (tid < (int)nb - 1) {
        const uint64_t q = ((uint64_t)(tid + 1) * S) / nb;
        s_spl[tid] = s.key[pad16((int)q)] + mn;
    }
    __syncthreads();
    if (tid == 0) {
        for (uint32_t i = 1; i + 1 < nb; ++i) {
            if (s_spl[i] <= s_spl[i - 1]) s_spl[i] = s_spl[i - 1] == ~0ull ? ~0ull : s_spl[i - 1] + 1;
        }
        // a heavy key that is the first splitter: isolate it from below too
        // (keys below it form bucket 0, the key itself bucket 1)
    }
    __syncthreads();
    uint64_t* out = splitters + (uint64_t)blockIdx.x * (MAX_BUCKETS - 1);
    for (int i = tid; i < MAX_BUCKETS - 1; i += NT) out[i] = i < (int)nb - 1 ? s_spl[i] : ~0ull;
}

__device__ __forceinline__ uint32_t bucket_of(const uint64_t* s_spl, uint64_t key, uint32_t nb) {
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t step = MAX_BUCKETS / 2; step >= 1; step >>= 1) {
        if (s_spl[pos + step - 1] <= key) pos += step;
    }
    return pos < nb - 1 ? pos : nb - 1;
}

// ---------------------------------------------------------------------------
// Histogram pass: rows per (bucket, chunk), bucket-major per region.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(PART_NT) k_hist(const Region* __restrict__ regions,
                                                  const Chunk* __restrict__ chunks,
                                                  const uint64_t* __restrict__ splitters,
                                                  uint32_t* __restrict__ hist) {
    __shared__ uint64_t s_spl[MAX_BUCKETS];
    __shared__ uint32_t s_hist[MAX_BUCKETS];
    const Chunk C = chunks[blockIdx.x];
    const Region R = regions[C.region];
    const int tid = threadIdx.x;
    for (int i = tid; i < MAX_BUCKETS; i += PART_NT) {
        s_spl[i] = i < MAX_BUCKETS - 1 ? splitters[(uint64_t)C.region * (MAX_BUCKETS - 1) + i] : ~0ull;
        s_hist[i] = 0;
    }
    __syncthreads();
    const uint64_t* kp = R.src.key;
    const uint64_t st = R.src.stride;
    for (uint32_t i = tid; i < C.n; i += PART_NT) {
        const uint64_t key = kp[(C.start + i) * st];
        atomicAdd(&s_hist[bucket_of(s_spl, key, R.nb)], 1u);
    }
    __syncthreads();
    for (uint32_t b = tid; b < R.nb; b += PART_NT)
        hist[R.hist_base + (uint64_t)b * R.n_chunks + C.idx] = s_hist[b];
}

// ---------------------------------------------------------------------------
// Scatter pass: stable partition of each chunk by bucket into a row-major
// buffer at the scanned offsets.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(PART_NT) k_scatter(const Region* __restrict__ regions,
                                                     const Chunk* __restrict__ chunks,
                                                     const uint64_t* __restrict__ splitters,
                                                     const uint64_t* __restrict__ offs,
                                                     uint64_t* __restrict__ dst, Layout L) {
    constexpr int NT = PART_NT, IPT = PART_IPT, NW = NT / 64;
    __shared__ uint64_t s_spl[MAX_BUCKETS];
    __shared__ uint64_t s_run[MAX_BUCKETS];
    __shared__ uint32_t s_cnt[NW * MAX_BUCKETS];
    __shared__ uint32_t s_tot[MAX_BUCKETS];
    const Chunk C = chunks[blockIdx.x];
    const Region R = regions[C.region];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint64_t rbase = offs[R.hist_base];
    for (int i = tid; i < MAX_BUCKETS; i += NT) {
        s_spl[i] = i < MAX_BUCKETS - 1 ? splitters[(uint64_t)C.region * (MAX_BUCKETS - 1) + i] : ~0ull;
        s_run[i] = i < (int)R.nb ? offs[R.hist_base + (uint64_t)i * R.n_chunks + C.idx] - rbase + R.out_pos : 0;
    }
    __syncthreads();
    const ColView V = R.src;
    const int dbits = bit_length(R.nb - 1);
    for (uint32_t t0 = 0; t0 < C.n; t0 += NT * IPT) {
        uint32_t* wc = s_cnt + w * MAX_BUCKETS;
        for (int i = lane; i < MAX_BUCKETS; i += 64) wc[i] = 0;
        uint32_t rank[IPT], dig[IPT];
        bool ok[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t i = t0 + (uint32_t)(w * 64 * IPT + j * 64 + lane);
            ok[j] = i < C.n;
            uint32_t d = 0;
            if (ok[j]) d = bucket_of(s_spl, V.key[(C.start + i) * V.stride], R.nb);
            const uint64_t active = __ballot(ok[j]);
            const uint64_t match = wave_match(d, dbits, active);
            const uint32_t before = __popcll(match & lt);
            uint32_t base = 0;
            if (ok[j]) {
                base = wc[d];
                if (before == 0) wc[d] = base + (uint32_t)__popcll(match);
            }
            rank[j] = base + before;
            dig[j] = d;
        }
        __syncthreads();
        // per bucket: exclusive scan over waves; s_tot = the tile's bucket total
        for (int b = tid; b < MAX_BUCKETS; b += NT) {
            uint32_t run = 0;
            for (int ww = 0; ww < NW; ++ww) {
                const uint32_t c = s_cnt[ww * MAX_BUCKETS + b];
                s_cnt[ww * MAX_BUCKETS + b] = run;
                run += c;
            }
            s_tot[b] = run;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (!ok[j]) continue;
            const uint32_t i = t0 + (uint32_t)(w * 64 * IPT + j * 64 + lane);
            const uint64_t dpos = s_run[dig[j]] + s_cnt[w * MAX_BUCKETS + dig[j]] + rank[j];
            const Agg a = load_agg(V, C.start + i);
            store_row(dst + dpos * (uint64_t)L.words, L, a);
        }
        __syncthreads();
        for (int b = tid; b < MAX_BUCKETS; b += NT) s_run[b] += s_tot[b];
        __syncthreads();
    }
}

// Bucket boundaries (region-relative) for the host: bstart[r][b], b = 0..nb.
__global__ void k_bucket_starts(const Region* __restrict__ regions, const uint64_t* __restrict__ offs,
                                const uint64_t* __restrict__ bs_base, uint64_t* __restrict__ bstart) {
    const Region R = regions[blockIdx.x];
    const uint64_t rbase = offs[R.hist_base];
    uint64_t* out = bstart + bs_base[blockIdx.x];
    for (uint32_t b = threadIdx.x; b <= R.nb; b += blockDim.x)
        out[b] = b < R.nb ? offs[R.hist_base + (uint64_t)b * R.n_chunks] - rbase : R.n;
}

// ---------------------------------------------------------------------------
// Leaf sort-reduce: load a key range (<= LEAF_CAP rows), sort it in LDS, and
// collapse equal adjacent keys into state rows written at out_pos of the
// temp buffer; counts[leaf] = number of groups.
// ---------------------------------------------------------------------------

struct LeafSmem {
    SortSmem<LEAF_NT, LEAF_IPT> sort;
    uint64_t mm[2 * LEAF_NT / 64];
    uint64_t pre_cnt[LEAF_NT];
    uint64_t pre_sum[LEAF_NT];
    int64_t pre_mn[LEAF_NT];
    int64_t pre_mx[LEAF_NT];
    double pre_fs[LEAF_NT];
    uint32_t pre_flags[LEAF_NT];  // bit0: thread has a head, bit1: thread has rows
    uint32_t scan_tmp[LEAF_NT / 64 + 1];
};

__global__ void __launch_bounds__(LEAF_NT) k_leaf(const Leaf* __restrict__ leaves, OutView temp,
                                                  uint32_t* __restrict__ counts) {
    constexpr int NT = LEAF_NT, IPT = LEAF_IPT;
    __shared__ LeafSmem s;
    const Leaf Lf = leaves[blockIdx.x];
    if (Lf.kind != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t n = (uint32_t)Lf.n;
    const ColView V = Lf.src;
    uint64_t k[IPT];
    uint32_t v[IPT];
    uint64_t mn = ~0ull, mx = 0ull;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t q = (uint32_t)(w * 64 * IPT + j * 64 + lane);
        v[j] = q;
        if (q < n) {
            k[j] = V.key[(uint64_t)q * V.stride];
            mn = k[j] < mn ? k[j] : mn;
            mx = k[j] > mx ? k[j] : mx;
        } else {
            k[j] = 0;
        }
    }
    block_minmax<NT>(mn, mx, s.mm);
    const uint64_t range = mx - mn;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t q = (uint32_t)(w * 64 * IPT + j * 64 + lane);
        k[j] = q < n ? k[j] - mn : range;
    }
    block_radix_sort<NT, IPT>(k, v, bit_length(range), s.sort);

    // Blocked arrangement: thread t owns sorted positions [t*IPT, t*IPT+IPT).
    const int p0 = tid * IPT;
    uint32_t nheads = 0;
    {
        uint64_t prev = p0 > 0 ? s.sort.key[pad16(p0 - 1)] : 0;
        for (int j = 0; j < IPT; ++j) {
            const int p = p0 + j;
            if (p >= (int)n) break;
            const uint64_t kk = s.sort.key[pad16(p)];
            if (p == 0 || kk != prev) ++nheads;
            prev = kk;
        }
    }
    uint32_t total;
    const uint32_t obase = block_exclusive_scan<NT>(nheads, s.scan_tmp, total);

    Agg acc;
    empty_agg(acc);
    bool have_head = false;
    uint32_t h = 0;
    uint64_t prev = p0 > 0 ? s.sort.key[pad16(p0 - 1)] : 0;
    int nrows = 0;
    for (int j = 0; j < IPT; ++j) {
        const int p = p0 + j;
        if (p >= (int)n) break;
        ++nrows;
        const uint64_t kk = s.sort.key[pad16(p)];
        const uint32_t row = s.sort.val[pad16(p)];
        Agg r;
        r.key = kk + mn;
        load_payload(V, row, r);
        const bool head = (p == 0) || (kk != prev);
        prev = kk;
        if (head) {
            if (!have_head) {
                s.pre_cnt[tid] = acc.cnt;
                s.pre_sum[tid] = acc.sum;
                s.pre_mn[tid] = acc.mn;
                s.pre_mx[tid] = acc.mx;
                s.pre_fs[tid] = acc.fs;
                have_head = true;
            } else {
                store_agg(temp, Lf.out_pos + obase + h - 1, acc);
            }
            acc = r;
            ++h;
        } else {
            combine(acc, r);
        }
    }
    if (!have_head) {
        s.pre_cnt[tid] = acc.cnt;
        s.pre_sum[tid] = acc.sum;
        s.pre_mn[tid] = acc.mn;
        s.pre_mx[tid] = acc.mx;
        s.pre_fs[tid] = acc.fs;
    }
    s.pre_flags[tid] = (have_head ? 1u : 0u) | (nrows > 0 ? 2u : 0u);
    __syncthreads();
    if (have_head) {
        // the last group of this thread continues into following threads up
        // to the next thread that starts a group
        for (int u = tid + 1; u < NT; ++u) {
            const uint32_t f = s.pre_flags[u];
            if (!(f & 2u)) break;
            Agg b;
            b.cnt = s.pre_cnt[u];
            b.sum = s.pre_sum[u];
            b.mn = s.pre_mn[u];
            b.mx = s.pre_mx[u];
            b.fs = s.pre_fs[u];
            combine(acc, b);
            if (f & 1u) break;
        }
        store_agg(temp, Lf.out_pos + obase + h - 1, acc);
    }
    if (tid == 0) counts[blockIdx.x] = total;
}

// ---------------------------------------------------------------------------
// Single-key leaves: every row has the same key; reduce in pieces, then
// combine the pieces' partials with a fixed tree.
// ---------------------------------------------------------------------------

template <int NT>
__device__ void block_reduce_agg(Agg& a, Agg* s_agg) {
    const int tid = threadIdx.x;
    s_agg[tid] = a;
    __syncthreads();
    for (int half = NT / 2; half >= 1; half >>= 1) {
        if (tid < half) combine(s_agg[tid], s_agg[tid + half]);
        __syncthreads();
    }
    a = s_agg[0];
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_single_partial(const Leaf* __restrict__ leaves,
                                                        const SinglePiece* __restrict__ pieces,
                                                        Agg* __restrict__ partials) {
    __shared__ Agg s_agg[256];
    const SinglePiece P = pieces[blockIdx.x];
    const ColView V = leaves[P.leaf].src;
    Agg a;
    empty_agg(a);
    for (uint32_t i = threadIdx.x; i < P.n; i += 256) {
        Agg r;
        load_payload(V, P.start + i, r);
        combine(a, r);
    }
    block_reduce_agg<256>(a, s_agg);
    if (threadIdx.x == 0) {
        a.key = V.key[P.start * V.stride];
        partials[P.slot] = a;
    }
}

__global__ void __launch_bounds__(256) k_single_final(const Leaf* __restrict__ leaves,
                                                      const Agg* __restrict__ partials, OutView temp,
                                                      uint32_t* __restrict__ counts) {
    __shared__ Agg s_agg[256];
    const Leaf Lf = leaves[blockIdx.x];
    if (Lf.kind != 1) return;
    Agg a;
    empty_agg(a);
    for (uint32_t i = threadIdx.x; i < Lf.single_count; i += 256) combine(a, partials[Lf.single_first + i]);
    block_reduce_agg<256>(a, s_agg);
    if (threadIdx.x == 0) {
        a.key = partials[Lf.single_first].key;
        store_agg(temp, Lf.out_pos, a);
        counts[blockIdx.x] = 1;
    }
}

// ---------------------------------------------------------------------------
// Merge of two sorted runs of unique keys with aggregation of equal keys
// (merge path; a split never separates an equal pair).  Partition p covers
// diagonals [p*MERGE_D, ...) and writes its groups at temp[p*MERGE_D ...].
// ---------------------------------------------------------------------------

__device__ __forceinline__ void merge_split(const ColView& A, uint64_t na, const ColView& B, uint64_t nb,
                                            uint64_t d, uint64_t& i_out, uint64_t& j_out) {
    uint64_t lo = d > nb ? d - nb : 0;
    uint64_t hi = d < na ? d : na;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (A.key[mid * A.stride] <= B.key[(d - 1 - mid) * B.stride]) lo = mid + 1;
        else hi = mid;
    }
    uint64_t i = lo, j = d - lo;
    if (i > 0 && j < nb && A.key[(i - 1) * A.stride] == B.key[j * B.stride]) ++j;
    i_out = i;
    j_out = j;
}

// Per-thread sub-range of a merge partition: thread t of partition p covers
// diagonals [p*MERGE_D + t*PER, ...).
struct MergeRange {
    uint64_t ia, ib, ja, jb;
};

__device__ __forceinline__ MergeRange merge_thread_range(const ColView& A, uint64_t na, const ColView& B,
                                                         uint64_t nb, uint64_t* s_i, uint64_t* s_j) {
    constexpr int NT = 256, PER = MERGE_D / NT;
    const int tid = threadIdx.x;
    const uint64_t total = na + nb;
    const uint64_t d0 = (uint64_t)blockIdx.x * MERGE_D;
    uint64_t d = d0 + (uint64_t)tid * PER;
    if (d > total) d = total;
    merge_split(A, na, B, nb, d, s_i[tid], s_j[tid]);
    if (tid == 0) {
        uint64_t de = d0 + MERGE_D;
        if (de > total) de = total;
        merge_split(A, na, B, nb, de, s_i[NT], s_j[NT]);
    }
    __syncthreads();
    MergeRange r;
    r.ia = s_i[tid];
    r.ib = s_i[tid + 1] > r.ia ? s_i[tid + 1] : r.ia;
    r.ja = s_j[tid];
    r.jb = s_j[tid + 1] > r.ja ? s_j[tid + 1] : r.ja;
    return r;
}

__device__ __forceinline__ uint32_t merge_count_range(const ColView& A, const ColView& B, const MergeRange& m) {
    uint32_t c = 0;
    uint64_t i = m.ia, j = m.ja;
    while (i < m.ib || j < m.jb) {
        if (j >= m.jb) ++i;
        else if (i >= m.ib) ++j;
        else {
            const uint64_t ka = A.key[i * A.stride], kb = B.key[j * B.stride];
            if (ka < kb) ++i;
            else if (kb < ka) ++j;
            else { ++i; ++j; }
        }
        ++c;
    }
    return c;
}

// Pass 1: groups produced by each partition.
__global__ void __launch_bounds__(256) k_merge_count(ColView A, uint64_t na, ColView B, uint64_t nb,
                                                     uint32_t* __restrict__ counts) {
    __shared__ uint64_t s_i[257], s_j[257];
    __shared__ uint32_t s_tmp[256 / 64 + 1];
    const MergeRange m = merge_thread_range(A, na, B, nb, s_i, s_j);
    const uint32_t c = merge_count_range(A, B, m);
    uint32_t tot;
    block_exclusive_scan<256>(c, s_tmp, tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// Pass 2: write each partition's groups at its scanned offset.
__global__ void __launch_bounds__(256) k_merge_write(ColView A, uint64_t na, ColView B, uint64_t nb,
                                                     const uint64_t* __restrict__ offs, OutView out) {
    __shared__ uint64_t s_i[257], s_j[257];
    __shared__ uint32_t s_tmp[256 / 64 + 1];
    const MergeRange m = merge_thread_range(A, na, B, nb, s_i, s_j);
    const uint32_t c = merge_count_range(A, B, m);
    uint32_t tot;
    const uint32_t base = block_exclusive_scan<256>(c, s_tmp, tot);
    uint64_t o = offs[blockIdx.x] + base;
    uint64_t i = m.ia, j = m.ja;
    while (i < m.ib || j < m.jb) {
        Agg r;
        if (j >= m.jb) { r = load_agg(A, i); ++i; }
        else if (i >= m.ib) { r = load_agg(B, j); ++j; }
        else {
            const uint64_t ka = A.key[i * A.stride], kb = B.key[j * B.stride];
            if (ka < kb) { r = load_agg(A, i); ++i; }
            else if (kb < ka) { r = load_agg(B, j); ++j; }
            else {
                r = load_agg(A, i);
                const Agg rb = load_agg(B, j);
                combine(r, rb);
                ++i;
                ++j;
            }
        }
        store_agg(out, o++, r);
    }
}

// Copy n rows between strided views, writing only below `cap`.
__global__ void __launch_bounds__(256) k_copy_rows(ColView src, uint64_t n, OutView dst, uint64_t cap) {
    const uint64_t lim = n < cap ? n : cap;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < lim; i += (uint64_t)gridDim.x * 256) {
        const Agg a = load_agg(src, i);
        store_agg(dst, i, a);
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 counts into uint64 offsets (three phases).
// ---------------------------------------------------------------------------

constexpr int SCAN_NT = 256;
constexpr int SCAN_IPT = 16;
constexpr int SCAN_TILE = SCAN_NT * SCAN_IPT;

__global__ void __launch_bounds__(SCAN_NT) k_scan_reduce(const uint32_t* __restrict__ in, uint64_t n,
                                                         uint64_t* __restrict__ tile_sums) {
    __shared__ uint64_t s[SCAN_NT];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint64_t acc = 0;
    for (int j = 0; j < SCAN_IPT; ++j) {
        const uint64_t i = base + (uint64_t)j * SCAN_NT + threadIdx.x;
        if (i < n) acc += in[i];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int half = SCAN_NT / 2; half >= 1; half >>= 1) {
        if ((int)threadIdx.x < half) s[threadIdx.x] += s[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = s[0];
}

// Single workgroup: exclusive scan of tile sums in place; total at [ntiles].
__global__ void __launch_bounds__(1024) k_scan_tiles(uint64_t* __restrict__ tile_sums, uint64_t ntiles) {
    __shared__ uint64_t s[1024];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t b0 = 0; b0 < ntiles; b0 += 1024) {
        const uint64_t i = b0 + threadIdx.x;
        const uint64_t x = i < ntiles ? tile_sums[i] : 0;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint64_t y = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < ntiles) tile_sums[i] = carry + s[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 0) carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sums[ntiles] = carry;
}

__global__ void __launch_bounds__(SCAN_NT) k_scan_final(const uint32_t* __restrict__ in, uint64_t n,
                                                        const uint64_t* __restrict__ tile_sums,
                                                        uint64_t* __restrict__ out) {
    __shared__ uint32_t s_tmp[SCAN_NT / 64 + 1];
    // blocked: thread t owns elements [t*IPT, t*IPT+IPT) of the tile
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_IPT;
    uint32_t loc[SCAN_IPT];
    uint32_t acc = 0;
    for (int j = 0; j < SCAN_IPT; ++j) {
        const uint64_t i = base + j;
        loc[j] = i < n ? in[i] : 0u;
        acc += loc[j];
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<SCAN_NT>(acc, s_tmp, tot);
    uint64_t run = tile_sums[blockIdx.x] + ex;
    for (int j = 0; j < SCAN_IPT; ++j) {
        const uint64_t i = base + j;
        if (i < n) out[i] = run;
        run += loc[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_NT - 1) out[n] = tile_sums[gridDim.x];
}

// ---------------------------------------------------------------------------
// Placement of gapped outputs: segment s (counts[s] rows at temp[src_pos])
// goes to dests[inst] at offs[s] - offs[first_seg[inst]].
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_compact(const Segment* __restrict__ segs, const uint32_t* __restrict__ counts,
                                                 const uint64_t* __restrict__ offs,
                                                 const uint32_t* __restrict__ first_seg,
                                                 const Dest* __restrict__ dests, ColView temp) {
    const Segment S = segs[blockIdx.x];
    const uint32_t c = counts[blockIdx.x];
    const Dest D = dests[S.inst];
    const uint64_t dst0 = offs[blockIdx.x] - offs[first_seg[S.inst]];
    for (uint32_t r = threadIdx.x; r < c; r += 256) {
        const uint64_t d = dst0 + r;
        if (d >= D.capacity) break;
        const Agg a = load_agg(temp, S.src_pos + r);
        store_agg(D.out, d, a);
    }
}

// n_groups per instance: offs[end] - offs[first].
__global__ void k_inst_totals(const uint64_t* __restrict__ offs, const uint32_t* __restrict__ first_seg,
                              uint32_t n_inst, uint64_t* __restrict__ totals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_inst) totals[i] = offs[first_seg[i + 1]] - offs[first_seg[i]];
}


// ---------------------------------------------------------------------------
// Composite keys (A int32, B int32): an order-preserving normalized key
// (Section 2.4: normalized keys compare as binary strings).  Flipping the sign
// bit maps signed order onto unsigned order.
// ---------------------------------------------------------------------------

__global__ void k_pack_pairs(const int32_t* __restrict__ a, const int32_t* __restrict__ b, uint64_t n,
                             uint64_t* __restrict__ keys) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        keys[i] = ((uint64_t)((uint32_t)a[i] ^ 0x80000000u) << 32) | (uint64_t)((uint32_t)b[i] ^ 0x80000000u);
}

__global__ void k_unpack_pairs(const uint64_t* __restrict__ keys, uint64_t n, int32_t* __restrict__ a,
                               int32_t* __restrict__ b) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const uint64_t k = keys[i];
        a[i] = (int32_t)((uint32_t)(k >> 32) ^ 0x80000000u);
        b[i] = (int32_t)((uint32_t)k ^ 0x80000000u);
    }
}

// Segment starts of a non-decreasing column: counts per chunk; *bad is set
// when a decreasing step is seen.
__global__ void __launch_bounds__(256) k_seg_count(const int32_t* __restrict__ a, uint64_t n, uint32_t chunk,
                                                   uint32_t* __restrict__ counts, uint32_t* __restrict__ bad) {
    __shared__ uint32_t s_tmp[256 / 64 + 1];
    const uint64_t c0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    uint32_t c = 0, b = 0;
    for (uint64_t i = c0 + threadIdx.x; i < c1; i += 256) {
        if (i == 0 || a[i] != a[i - 1]) ++c;
        if (i > 0 && a[i] < a[i - 1]) b = 1;
    }
    uint32_t tot;
    block_exclusive_scan<256>(c, s_tmp, tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
    if (b) atomicOr(bad, 1u);
}

__global__ void __launch_bounds__(256) k_seg_write(const int32_t* __restrict__ a, uint64_t n, uint32_t chunk,
                                                   const uint64_t* __restrict__ offs, uint64_t* __restrict__ starts) {
    __shared__ uint32_t s_tmp[256 / 64 + 1];
    const uint64_t c0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    // thread t scans a contiguous sub-range so that starts come out in order
    const uint64_t per = (chunk + 255) / 256;
    const uint64_t t0 = c0 + threadIdx.x * per;
    const uint64_t t1 = t0 + per < c1 ? t0 + per : c1;
    uint32_t c = 0;
    for (uint64_t i = t0; i < t1; ++i)
        if (i == 0 || a[i] != a[i - 1]) ++c;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<256>(c, s_tmp, tot);
    uint64_t o = offs[blockIdx.x] + ex;
    for (uint64_t i = t0; i < t1; ++i)
        if (i == 0 || a[i] != a[i - 1]) starts[o++] = i;
}

// ---------------------------------------------------------------------------
// Host-side launch wrappers
// ---------------------------------------------------------------------------

void launch_sample(const Region* regions, uint32_t n_regions, uint64_t* splitters, hipStream_t st) {
    hipLaunchKernelGGL(k_sample, dim3(n_regions), dim3(LEAF_NT), 0, st, regions, splitters);
}
void launch_hist(const Region* regions, const Chunk* chunks, uint32_t n_chunks, const uint64_t* splitters,
                 uint32_t* hist, hipStream_t st) {
    hipLaunchKernelGGL(k_hist, dim3(n_chunks), dim3(PART_NT), 0, st, regions, chunks, splitters, hist);
}
void launch_scatter(const Region* regions, const Chunk* chunks, uint32_t n_chunks, const uint64_t* splitters,
                    const uint64_t* offs, uint64_t* dst, Layout L, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter, dim3(n_chunks), dim3(PART_NT), 0, st, regions, chunks, splitters, offs, dst, L);
}
void launch_bucket_starts(const Region* regions, uint32_t n_regions, const uint64_t* offs, const uint64_t* bs_base,
                          uint64_t* bstart, hipStream_t st) {
    hipLaunchKernelGGL(k_bucket_starts, dim3(n_regions), dim3(256), 0, st, regions, offs, bs_base, bstart);
}
void launch_leaf(const Leaf* leaves, uint32_t n_leaves, OutView temp, uint32_t* counts, hipStream_t st) {
    hipLaunchKernelGGL(k_leaf, dim3(n_leaves), dim3(LEAF_NT), 0, st, leaves, temp, counts);
}
void launch_single(const Leaf* leaves, uint32_t n_leaves, const SinglePiece* pieces, uint32_t n_pieces,
                   void* partials, OutView temp, uint32_t* counts, hipStream_t st) {
    hipLaunchKernelGGL(k_single_partial, dim3(n_pieces), dim3(256), 0, st, leaves, pieces, (Agg*)partials);
    hipLaunchKernelGGL(k_single_final, dim3(n_leaves), dim3(256), 0, st, leaves, (const Agg*)partials, temp, counts);
}
size_t single_partial_bytes() { return sizeof(Agg); }
uint64_t merge_parts(uint64_t na, uint64_t nb) { return (na + nb + MERGE_D - 1) / MERGE_D; }
void launch_merge_count(ColView A, uint64_t na, ColView B, uint64_t nb, uint32_t* counts, hipStream_t st) {
    const uint64_t parts = merge_parts(na, nb);
    if (parts == 0) return;
    hipLaunchKernelGGL(k_merge_count, dim3((uint32_t)parts), dim3(256), 0, st, A, na, B, nb, counts);
}
void launch_merge_write(ColView A, uint64_t na, ColView B, uint64_t nb, const uint64_t* offs, OutView out,
                        hipStream_t st) {
    const uint64_t parts = merge_parts(na, nb);
    if (parts == 0) return;
    hipLaunchKernelGGL(k_merge_write, dim3((uint32_t)parts), dim3(256), 0, st, A, na, B, nb, offs, out);
}
void launch_copy_rows(ColView src, uint64_t n, OutView dst, uint64_t cap, hipStream_t st) {
    const uint64_t lim = n < cap ? n : cap;
    if (lim == 0) return;
    uint64_t g = (lim + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_copy_rows, dim3((uint32_t)g), dim3(256), 0, st, src, n, dst, cap);
}
uint64_t scan_tiles(uint64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }
// offs must hold n+1 entries, tile_sums scan_tiles(n)+1 entries.
void launch_scan(const uint32_t* in, uint64_t n, uint64_t* tile_sums, uint64_t* offs, hipStream_t st) {
    const uint64_t t = scan_tiles(n);
    if (t == 0) {
        hipMemsetAsync(offs, 0, sizeof(uint64_t), st);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)t), dim3(SCAN_NT), 0, st, in, n, tile_sums);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, tile_sums, t);
    hipLaunchKernelGGL(k_scan_final, dim3((uint32_t)t), dim3(SCAN_NT), 0, st, in, n, tile_sums, offs);
}
void launch_compact(const Segment* segs, uint32_t n_segs, const uint32_t* counts, const uint64_t* offs,
                    const uint32_t* first_seg, const Dest* dests, ColView temp, hipStream_t st) {
    if (n_segs == 0) return;
    hipLaunchKernelGGL(k_compact, dim3(n_segs), dim3(256), 0, st, segs, counts, offs, first_seg, dests, temp);
}
static dim3 grid_rows(uint64_t n) {
    uint64_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    return dim3((uint32_t)(g ? g : 1));
}
void launch_pack_pairs(const int32_t* a, const int32_t* b, uint64_t n, uint64_t* keys, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_pack_pairs, grid_rows(n), dim3(256), 0, st, a, b, n, keys);
}
void launch_unpack_pairs(const uint64_t* keys, uint64_t n, int32_t* a, int32_t* b, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_unpack_pairs, grid_rows(n), dim3(256), 0, st, keys, n, a, b);
}
void launch_seg_count(const int32_t* a, uint64_t n, uint32_t chunk, uint32_t* counts, uint32_t* bad,
                      hipStream_t st) {
    const uint64_t g = (n + chunk - 1) / chunk;
    if (!g) return;
    hipLaunchKernelGGL(k_seg_count, dim3((uint32_t)g), dim3(256), 0, st, a, n, chunk, counts, bad);
}
void launch_seg_write(const int32_t* a, uint64_t n, uint32_t chunk, const uint64_t* offs, uint64_t* starts,
                      hipStream_t st) {
    const uint64_t g = (n + chunk - 1) / chunk;
    if (!g) return;
    hipLaunchKernelGGL(k_seg_write, dim3((uint32_t)g), dim3(256), 0, st, a, n, chunk, offs, starts);
}
void launch_inst_totals(const uint64_t* offs, const uint32_t* first_seg, uint32_t n_inst, uint64_t* totals,
                        hipStream_t st) {
    if (n_inst == 0) return;
    hipLaunchKernelGGL(k_inst_totals, dim3((n_inst + 255) / 256), dim3(256), 0, st, offs, first_seg, n_inst, totals);
}

}  // namespace isa
