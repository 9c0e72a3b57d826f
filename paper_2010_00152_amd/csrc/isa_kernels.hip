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

#include <mutex>

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

// ---------------------------------------------------------------------------
// Segmented scan of per-thread aggregates across a workgroup, for groups that
// span threads.  Thread t contributes y_t; a thread with `start` set begins a
// segment.  Inside a wave the inclusive scan R_t = start_t ? y_t :
// R_{t-1} + y_t takes DPP lane moves (row shifts by 1, 2, 4 and 8 lanes, then
// the broadcasts of lanes 15 and 31 to the rows after them); across waves the
// waves' last lanes go through LDS.  Each thread gets R_{t-1}, the open
// segment's aggregate at the end of the thread before it (empty for t = 0),
// and R_t.  The combination order is fixed, so results repeat exactly.
// ---------------------------------------------------------------------------

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROW_MASK, 0xf, false);
    return (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_agg(const Agg& r, uint32_t f, Agg& t, uint32_t& tf) {
    t.cnt = dpp_u64<CTRL, ROW_MASK>(r.cnt);
    t.sum = dpp_u64<CTRL, ROW_MASK>(r.sum);
    t.mn = (int64_t)dpp_u64<CTRL, ROW_MASK>((uint64_t)r.mn);
    t.mx = (int64_t)dpp_u64<CTRL, ROW_MASK>((uint64_t)r.mx);
    t.fs = __longlong_as_double((long long)dpp_u64<CTRL, ROW_MASK>((uint64_t)__double_as_longlong(r.fs)));
    tf = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)f, CTRL, ROW_MASK, 0xf, false);
}

// One step: lanes with `take` add the moved partial (the lanes before them)
// to their own unless their segment already started.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_step(Agg& r, uint32_t& f, bool take) {
    Agg t;
    uint32_t tf;
    dpp_agg<CTRL, ROW_MASK>(r, f, t, tf);
    if (take) {
        if (!f) {
            combine(t, r);
            r.cnt = t.cnt;
            r.sum = t.sum;
            r.mn = t.mn;
            r.mx = t.mx;
            r.fs = t.fs;
        }
        f |= tf;
    }
}

template <int NT>
__device__ __forceinline__ void seg_scan_agg(const Agg& y, bool start, Agg& prev, Agg& incl, Agg* s_w,
                                             uint32_t* s_wf) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, rl = lane & 15;
    Agg r = y;
    uint32_t f = start ? 1u : 0u;
    // DPP controls (gfx9): row_shr:n = 0x110 + n, wave_shr:1 = 0x138,
    // row_bcast:15 = 0x142 (rows 1 and 3), row_bcast:31 = 0x143 (rows 2 and 3)
    seg_step<0x111, 0xf>(r, f, rl >= 1);
    seg_step<0x112, 0xf>(r, f, rl >= 2);
    seg_step<0x114, 0xf>(r, f, rl >= 4);
    seg_step<0x118, 0xf>(r, f, rl >= 8);
    seg_step<0x142, 0xa>(r, f, (lane & 31) >= 16);
    seg_step<0x143, 0xc>(r, f, lane >= 32);
    if (lane == 63) {
        s_w[w] = r;
        s_wf[w] = f;
    }
    // the thread before: one lane down the wave (lane 0 takes the waves before)
    Agg p;
    uint32_t pf;
    dpp_agg<0x138, 0xf>(r, f, p, pf);
    __syncthreads();
    // a segment open at the wave's start continues from the waves before
    Agg c;
    empty_agg(c);
    for (int w2 = w - 1; w2 >= 0; --w2) {
        Agg t = s_w[w2];
        combine(t, c);
        c = t;
        if (s_wf[w2]) break;
    }
    if (!f) {
        Agg t = c;
        combine(t, r);
        r = t;
    }
    if (lane == 0) {
        p = c;
    } else if (!pf) {
        Agg t = c;
        combine(t, p);
        p = t;
    }
    prev = p;
    incl = r;
    __syncthreads();  // s_w is reused by the next call
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

__device__ __forceinline__ int pad16(int p) { return p + (p >> 4); }

// ---------------------------------------------------------------------------
// Block radix sort with per-thread digit counters.  Items are in registers,
// thread t holding logical items t*IPT .. t*IPT+IPT-1.  Each pass ranks one
// 4-bit digit: every thread counts its own items per digit in a private LDS
// column (no conflicts between threads, order kept within a thread), one
// block-wide scan over the counters in digit-major, thread-minor order gives
// every (digit, thread) its base, and items move to base + local rank.  The
// sort is stable, so passes go from the lowest digit up.  Sorted pairs end in
// s.key/s.val at pad16(position).
// ---------------------------------------------------------------------------

// (4-bit digits keep the counters at 8 KB: with them a leaf workgroup takes
// 52.6 KB of LDS and fits three to a CU, against two with 5-bit digits; the
// extra pass costs less than the occupancy gains, 100M-row leaf launch
// 3.77 -> 3.0 ms.)
constexpr int CNT_BITS = 4;
constexpr int CNT_DIGITS = 1 << CNT_BITS;

// Key bits (below the range's top) that leaf sorts and splitter samples order
// first; a leaf re-sorts at full width when two distinct keys share them.
constexpr int LEAF_TRUNC = 30;
// Key bits (below the range's top) that a leaf sorts on; distinct keys that
// share them are put in order afterwards in runs of at most LEAF_FIX_MAX rows.
constexpr int LEAF_SORT_BITS = 24;
constexpr int LEAF_FIX_MAX = 512;
constexpr int LEAF_FIX_RUNS = 32;

template <int NT, int IPT>
struct CSortSmem {
    static constexpr int N = NT * IPT;
    static constexpr int NP = N + N / 16;
    uint64_t key[NP];
    uint16_t val[NP];
    alignas(16) uint16_t cnt[CNT_DIGITS * NT];
    uint32_t tmp[NT / 64 + 1];
};

// Exclusive block scan with one barrier: every thread sums the wave totals
// itself.  s_tmp (NT/64 words) must not be rewritten before a later barrier.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan_1b(uint32_t x, uint32_t* s_tmp, uint32_t& total) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_inclusive_scan(x);
    if (lane == 63) s_tmp[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint32_t t = s_tmp[i];
        before += i < w ? t : 0u;
        all += t;
    }
    total = all;
    return before + inc - x;
}

// IPTC <= IPT items per thread take part (thread t: items t*IPTC ..
// t*IPTC+IPTC-1).  The count is a compile-time constant so that every loop
// over the items is straight-line code: a wave's LDS operations of all its
// items are in flight together instead of one item per round trip.
template <int NT, int IPT, int IPTC = IPT>
__device__ void block_sort_cnt(uint64_t (&k)[IPT], uint16_t (&v)[IPT], int lo_bit, int hi_bit,
                               CSortSmem<NT, IPT>& s) {
    static_assert(IPTC <= IPT, "active items per thread");
    constexpr int ipt = IPTC;
    static_assert((CNT_DIGITS * NT * 2) % (16 * NT) == 0, "counter zeroing layout");
    constexpr int ZERO4 = CNT_DIGITS * NT * 2 / 16 / NT;  // uint4 stores per thread
    constexpr int SEG = CNT_DIGITS;                       // counters scanned per thread
    const int tid = threadIdx.x;
    if (lo_bit >= hi_bit) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (j < ipt) {
                s.key[pad16(tid * ipt + j)] = k[j];
                s.val[pad16(tid * ipt + j)] = v[j];
            }
        }
        __syncthreads();
        return;
    }
    uint4* c4 = reinterpret_cast<uint4*>(s.cnt);
    // thread t's counter of digit d, cnt[d*NT + t], is half (t & 1) of a word
    uint32_t* cw = reinterpret_cast<uint32_t*>(s.cnt);
    const uint32_t half = (uint32_t)(tid & 1) * 16u;
    static_assert(NT % 2 == 0 && SEG % 8 == 0, "counter word and vector layout");
    for (int shift = lo_bit; shift < hi_bit; shift += CNT_BITS) {
        const int dbits = hi_bit - shift < CNT_BITS ? hi_bit - shift : CNT_BITS;
        const uint32_t mask = (1u << dbits) - 1u;
        const bool last = shift + CNT_BITS >= hi_bit;
#pragma unroll
        for (int i = 0; i < ZERO4; ++i) c4[i * NT + tid] = make_uint4(0, 0, 0, 0);
        __syncthreads();
        // the item's rank among the thread's earlier items of its digit: the
        // counter's old value, from LDS atomics issued back to back (a
        // wave's LDS operations complete in order)
        uint32_t loc[IPT], dg[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (j < ipt) {
                const uint32_t d = (uint32_t)(k[j] >> shift) & mask;
                dg[j] = d;
                loc[j] = (atomicAdd(&cw[(d * NT + tid) >> 1], 1u << half) >> half) & 0xffffu;
            }
        }
        __syncthreads();
        // scan the counters in memory order (digit-major, thread-minor),
        // eight per 16-byte load
        uint4* seg4 = reinterpret_cast<uint4*>(s.cnt + tid * SEG);
        uint4 q[SEG / 8];
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < SEG / 8; ++i) {
            q[i] = seg4[i];
            const uint32_t h = q[i].x + q[i].y + q[i].z + q[i].w;  // two 16-bit sums, no carry (<= N)
            sum += (h & 0xffffu) + (h >> 16);
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan_1b<NT>(sum, s.tmp, total);
        auto pre2 = [&](uint32_t& wd) {
            // the word's two counters become their exclusive prefixes
            const uint32_t lo = wd & 0xffffu, hi = wd >> 16;
            wd = run | ((run + lo) << 16);
            run += lo + hi;
        };
#pragma unroll
        for (int i = 0; i < SEG / 8; ++i) {
            pre2(q[i].x);
            pre2(q[i].y);
            pre2(q[i].z);
            pre2(q[i].w);
            seg4[i] = q[i];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (j < ipt) {
                const int pos = (int)s.cnt[dg[j] * NT + tid] + (int)loc[j];
                s.key[pad16(pos)] = k[j];
                s.val[pad16(pos)] = v[j];
            }
        }
        __syncthreads();
        if (!last) {
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
                if (j < ipt) {
                    k[j] = s.key[pad16(tid * ipt + j)];
                    v[j] = s.val[pad16(tid * ipt + j)];
                }
            }
        }
    }
}

// Move items loaded warp-striped (coalesced: item j of lane l in wave w is row
// w*64*IPT + j*64 + l) into blocked order (thread t holds rows t*IPT ..
// t*IPT+IPT-1) through LDS, so the first sort pass sees rows in row order and
// padding rows (beyond n) stay after every real row.
template <int NT, int IPT, int IPTC = IPT>
__device__ void striped_to_blocked(uint64_t (&k)[IPT], uint16_t (&v)[IPT], CSortSmem<NT, IPT>& s) {
    constexpr int ipt = IPTC;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int q = w * 64 * IPT + j * 64 + lane;
        s.key[pad16(q)] = k[j];
        s.val[pad16(q)] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        if (j < ipt) {
            k[j] = s.key[pad16(tid * ipt + j)];
            v[j] = s.val[pad16(tid * ipt + j)];
        }
    }
    __syncthreads();
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

// Row at the middle of stratum q of S equal strata of n rows:
// floor((2q + 1) n / (2S)).  The product fits 64 bits for every n below 2^48
// (q < S <= 2^15), and a power-of-two S divides by a shift; otherwise the
// library's 64-bit or, beyond 2^48 rows, 128-bit division (slow on the GPU)
// is used.
__device__ __forceinline__ uint64_t stratum_row(uint64_t q, uint64_t n, uint64_t S) {
    const uint64_t den = 2 * S;
    if (n < (1ull << 48)) {
        const uint64_t num = (2 * q + 1) * n;
        return (den & (den - 1)) == 0 ? num >> __builtin_ctzll(den) : num / den;
    }
    return (uint64_t)(((unsigned __int128)(2 * q + 1) * n) / den);
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
    __shared__ CSortSmem<NT, IPT> s;
    __shared__ uint64_t s_mm[2 * NT / 64];
    const Region R = regions[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t S = R.n < (uint64_t)SAMPLE_N ? R.n : (uint64_t)SAMPLE_N;
    uint64_t k[IPT];
    uint16_t v[IPT];
    uint64_t mn = ~0ull, mx = 0ull;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint64_t q = (uint64_t)(w * 64 * IPT + j * 64 + lane);
        v[j] = (uint16_t)q;
        if (q < S) {
            const uint64_t pos = stratum_row(q, R.n, S);
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
    striped_to_blocked<NT, IPT>(k, v, s);
    // quantiles need only the order of the top LEAF_TRUNC bits: keys that
    // agree on them may stay unordered among themselves (any increasing
    // splitters are valid; the fix-up below makes them strictly increasing)
    const int nbits = bit_length(range);
    block_sort_cnt<NT, IPT>(k, v, nbits > LEAF_TRUNC ? nbits - LEAF_TRUNC : 0, nbits, s);
    __shared__ uint64_t s_spl[MAX_BUCKETS];
    const uint32_t nb = R.nb;
    for (int i = tid; i < (int)nb - 1; i += NT) {
        const uint64_t q = ((uint64_t)(i + 1) * S) / nb;
        s_spl[i] = s.key[pad16((int)q)] + mn;
    }
    __syncthreads();
    // Strictly increasing splitters: t[i] = max(s[i], t[i-1] + 1), saturating
    // at the largest key value, which is t[i] = max over j <= i of
    // s[j] + (i - j); a doubling scan over the nb-1 splitters (one per thread)
    // computes it in log2(nb) steps.
    {
        static_assert(MAX_BUCKETS <= NT, "one splitter per thread");
        const int m = (int)nb - 1;
        uint64_t t = tid < m ? s_spl[tid] : 0;
        for (int d = 1; d < m; d <<= 1) {
            const uint64_t prev = tid >= d && tid < m ? s_spl[tid - d] : 0;
            __syncthreads();
            if (tid >= d && tid < m) {
                const uint64_t c = prev + (uint64_t)d;
                const uint64_t sat = c < prev ? ~0ull : c;
                t = sat > t ? sat : t;
                s_spl[tid] = t;
            }
            __syncthreads();
        }
    }
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

__device__ __forceinline__ void hist_chunk(const Region& R, const Chunk& C, const uint64_t* __restrict__ splitters,
                                           uint32_t* __restrict__ hist, uint64_t* s_spl, uint32_t* s_hist);

__global__ void __launch_bounds__(PART_NT) k_hist(const Region* __restrict__ regions,
                                                  const Chunk* __restrict__ chunks,
                                                  const uint64_t* __restrict__ splitters,
                                                  uint32_t* __restrict__ hist) {
    __shared__ uint64_t s_spl[MAX_BUCKETS];
    __shared__ uint32_t s_hist[MAX_BUCKETS];
    const Chunk C = chunks[blockIdx.x];
    hist_chunk(regions[C.region], C, splitters, hist, s_spl, s_hist);
}

// The histogram of one batch of run generation, which also sets the batch up
// for the launches after it: the region descriptor (passed by value) is
// stored for them and the batch's control block is cleared.
__global__ void __launch_bounds__(PART_NT) k_hist_batch(Region r, Region* __restrict__ reg,
                                                        uint64_t* __restrict__ ctl, uint32_t ctl_words,
                                                        const Chunk* __restrict__ chunks,
                                                        const uint64_t* __restrict__ splitters,
                                                        uint32_t* __restrict__ hist) {
    __shared__ uint64_t s_spl[MAX_BUCKETS];
    __shared__ uint32_t s_hist[MAX_BUCKETS];
    for (uint32_t i = blockIdx.x * PART_NT + threadIdx.x; i < ctl_words; i += gridDim.x * PART_NT) ctl[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *reg = r;
    hist_chunk(r, chunks[blockIdx.x], splitters, hist, s_spl, s_hist);
}

__device__ __forceinline__ void hist_chunk(const Region& R, const Chunk& C, const uint64_t* __restrict__ splitters,
                                           uint32_t* __restrict__ hist, uint64_t* s_spl, uint32_t* s_hist) {
    const int tid = threadIdx.x;
    for (int i = tid; i < MAX_BUCKETS; i += PART_NT) {
        s_spl[i] = i < MAX_BUCKETS - 1 ? splitters[(uint64_t)C.region * (MAX_BUCKETS - 1) + i] : ~0ull;
        s_hist[i] = 0;
    }
    __syncthreads();
    const uint64_t* kp = R.src.key;
    const uint64_t st = R.src.stride;
    // eight keys in flight per thread
    constexpr int HL = 8;
    for (uint32_t i0 = tid; i0 < C.n; i0 += PART_NT * HL) {
        uint64_t kk[HL];
#pragma unroll
        for (int q = 0; q < HL; ++q) {
            const uint32_t i = i0 + (uint32_t)q * PART_NT;
            if (i < C.n) kk[q] = kp[(C.start + i) * st];
        }
#pragma unroll
        for (int q = 0; q < HL; ++q) {
            const uint32_t i = i0 + (uint32_t)q * PART_NT;
            if (i < C.n) atomicAdd(&s_hist[bucket_of(s_spl, kk[q], R.nb)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t b = tid; b < R.nb; b += PART_NT)
        hist[R.hist_base + (uint64_t)b * R.n_chunks + C.idx] = s_hist[b];
}

// ---------------------------------------------------------------------------
// Scatter pass: stable partition of each chunk by bucket into a row-major
// buffer at the scanned offsets.  A tile's rows are first ranked into bucket
// order in LDS (row index and bucket per sorted slot); consecutive threads
// then move consecutive rows of one bucket, so the stores of a wave fill
// contiguous spans of the destination instead of one line per lane.
// ---------------------------------------------------------------------------

// SW > 0: rows of at most SW words are also loaded with the keys (coalesced)
// into LDS in input order and move from there; SW = 0: they are gathered
// from the source in bucket order.
template <int SW, int IPT>
__global__ void __launch_bounds__(PART_NT) k_scatter(const Region* __restrict__ regions,
                                                     const Chunk* __restrict__ chunks,
                                                     const uint64_t* __restrict__ splitters,
                                                     const uint64_t* __restrict__ offs,
                                                     uint64_t* __restrict__ dst, Layout L,
                                                     const uint32_t* __restrict__ hist_self,
                                                     uint64_t* __restrict__ offs_out) {
    constexpr int NT = PART_NT, NW = NT / 64, TILE = NT * IPT;
    static_assert(TILE <= 65536, "tile slots are 16-bit");
    static_assert(MAX_BUCKETS == NT, "one thread per bucket in the tile scan");
    __shared__ uint64_t s_rows[SW > 0 ? TILE * SW : 1];
    __shared__ uint64_t s_spl[MAX_BUCKETS];
    __shared__ uint64_t s_run[MAX_BUCKETS];
    __shared__ uint32_t s_cnt[NW * MAX_BUCKETS];
    __shared__ uint32_t s_tot[MAX_BUCKETS];
    __shared__ uint32_t s_lstart[MAX_BUCKETS];
    __shared__ uint32_t s_tmp[NT / 64 + 1];
    __shared__ uint16_t s_src[TILE];
    __shared__ uint8_t s_dig[TILE];
    const Chunk C = chunks[blockIdx.x];
    const Region R = regions[C.region];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int i = tid; i < MAX_BUCKETS; i += NT)
        s_spl[i] = i < MAX_BUCKETS - 1 ? splitters[(uint64_t)C.region * (MAX_BUCKETS - 1) + i] : ~0ull;
    if (hist_self) {
        // no separate scan: thread b sums bucket b over all chunks of the
        // region and over its chunks before this one; a scan over buckets
        // gives the bucket starts.  The region-relative offsets go to
        // offs_out for the leaves.
        uint32_t tot = 0, before = 0;
        if (tid < (int)R.nb) {
            const uint32_t* hb = hist_self + R.hist_base + (uint64_t)tid * R.n_chunks;
            uint32_t c = 0;
            if ((((uintptr_t)hb) & 15) == 0) {
                // four chunks per 16-byte load, several loads in flight
                const uint4* h4 = reinterpret_cast<const uint4*>(hb);
                const uint32_t n4 = R.n_chunks / 4;
#pragma unroll 8
                for (uint32_t q = 0; q < n4; ++q) {
                    const uint4 h = h4[q];
                    const uint32_t c0 = 4 * q;
                    tot += h.x + h.y + h.z + h.w;
                    before += (c0 < C.idx ? h.x : 0u) + (c0 + 1 < C.idx ? h.y : 0u) + (c0 + 2 < C.idx ? h.z : 0u) +
                              (c0 + 3 < C.idx ? h.w : 0u);
                }
                c = 4 * n4;
            }
            for (; c < R.n_chunks; ++c) {
                const uint32_t h = hb[c];
                tot += h;
                before += c < C.idx ? h : 0u;
            }
        }
        uint32_t all;
        const uint32_t base = block_exclusive_scan<NT>(tot, s_tmp, all);
        if (tid < (int)R.nb) {
            s_run[tid] = (uint64_t)(base + before) + R.out_pos;
            offs_out[R.hist_base + (uint64_t)tid * R.n_chunks + C.idx] = base + before;
        } else {
            s_run[tid] = 0;
        }
    } else {
        const uint64_t rbase = offs[R.hist_base];
        for (int i = tid; i < MAX_BUCKETS; i += NT)
            s_run[i] = i < (int)R.nb ? offs[R.hist_base + (uint64_t)i * R.n_chunks + C.idx] - rbase + R.out_pos : 0;
    }
    __syncthreads();
    const ColView V = R.src;
    const int dbits = bit_length(R.nb - 1);
    for (uint32_t t0 = 0; t0 < C.n; t0 += TILE) {
        const uint32_t tn = C.n - t0 < (uint32_t)TILE ? C.n - t0 : (uint32_t)TILE;
        uint32_t* wc = s_cnt + w * MAX_BUCKETS;
        for (int i = lane; i < MAX_BUCKETS; i += 64) wc[i] = 0;
        uint32_t rank[IPT], dig[IPT];
        bool ok[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t i = (uint32_t)(w * 64 * IPT + j * 64 + lane);
            ok[j] = i < tn;
            uint32_t d = 0;
            if (ok[j]) {
                if (SW > 0) {
                    const Agg a = load_agg(V, C.start + t0 + i);
                    store_row(s_rows + i * (uint32_t)L.words, L, a);
                    d = bucket_of(s_spl, a.key, R.nb);
                } else {
                    d = bucket_of(s_spl, V.key[(C.start + t0 + i) * V.stride], R.nb);
                }
            }
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
        {
            // bucket b (thread b): exclusive scan over waves, tile total, and
            // the bucket's first slot in the tile's bucket order
            uint32_t run = 0;
            for (int ww = 0; ww < NW; ++ww) {
                const uint32_t c = s_cnt[ww * MAX_BUCKETS + tid];
                s_cnt[ww * MAX_BUCKETS + tid] = run;
                run += c;
            }
            s_tot[tid] = run;
            uint32_t all;
            s_lstart[tid] = block_exclusive_scan<NT>(run, s_tmp, all);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (!ok[j]) continue;
            const uint32_t slot = s_lstart[dig[j]] + s_cnt[w * MAX_BUCKETS + dig[j]] + rank[j];
            s_src[slot] = (uint16_t)(w * 64 * IPT + j * 64 + lane);
            s_dig[slot] = (uint8_t)dig[j];
        }
        __syncthreads();
        for (uint32_t x = tid; x < tn; x += NT) {
            const uint32_t d = s_dig[x];
            const uint64_t dpos = s_run[d] + (x - s_lstart[d]);
            if (SW > 0) {
                const uint64_t* r = s_rows + (uint32_t)s_src[x] * (uint32_t)L.words;
                uint64_t* o = dst + dpos * (uint64_t)L.words;
#pragma unroll
                for (int q = 0; q < SW; ++q)
                    if (q < L.words) o[q] = r[q];
            } else {
                const Agg a = load_agg(V, C.start + t0 + s_src[x]);
                store_row(dst + dpos * (uint64_t)L.words, L, a);
            }
        }
        __syncthreads();
        s_run[tid] += s_tot[tid];
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

// ---------------------------------------------------------------------------
// Chained prefix over workgroups in ticket order (decoupled look-back): a
// workgroup publishes its own count as soon as it is known, then sums its
// predecessors' counts back to the nearest published inclusive prefix.
// Tickets are taken at workgroup start, so every predecessor has already
// started.  status[i] = 0 (not published), ST_AGG|count, or ST_PRE|inclusive.
// A wait that exceeds LOOKBACK_SPINS sets *err and gives up, so every wait
// ends; the host then reports the call as failed.
// ---------------------------------------------------------------------------

constexpr uint64_t ST_AGG = 1ull << 62;
constexpr uint64_t ST_PRE = 2ull << 62;
constexpr uint64_t ST_VAL = (1ull << 62) - 1;
constexpr uint32_t LOOKBACK_SPINS = 1u << 22;

// Status words are the only data one workgroup reads from another here, so
// relaxed device-scope atomics suffice (coherent across the chip without the
// cache writeback/invalidate that release/acquire ordering would add).
__device__ __forceinline__ void st_publish(uint64_t* p, uint64_t w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t st_read(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Called by all 64 lanes of one wave (i and first uniform).  Returns the
// exclusive prefix of item i over items first..i-1 and publishes the
// inclusive prefix of item i.  The wave reads 64 predecessors' status words
// at a time and sums back to the nearest published inclusive prefix.
__device__ uint64_t chained_prefix(uint64_t* status, uint32_t i, uint32_t first, uint64_t count, uint32_t* err) {
    const int lane = threadIdx.x & 63;
    if (i == first) {
        if (lane == 0) st_publish(&status[i], ST_PRE | count);
        return 0;
    }
    if (lane == 0) st_publish(&status[i], ST_AGG | count);
    uint64_t sum = 0;
    int64_t top = (int64_t)i - 1;
    uint32_t spins = 0;
    for (;;) {
        const int64_t j = top - lane;
        // items before `first` read as an inclusive prefix of zero
        const uint64_t w = j >= (int64_t)first ? st_read(&status[j]) : ST_PRE;
        const uint32_t flag = (uint32_t)(w >> 62);
        const uint64_t pre_mask = __ballot(flag == 2);
        const uint64_t zero_mask = __ballot(flag == 0);
        const int nearest = pre_mask ? __ffsll((long long)pre_mask) - 1 : 64;
        const uint64_t needed = nearest >= 63 ? ~0ull : ((1ull << (nearest + 1)) - 1ull);
        if (zero_mask & needed) {
            if (++spins >= LOOKBACK_SPINS) {
                if (lane == 0) atomicOr(err, 1u);
                __threadfence();  // the error bit is visible before this item's prefix
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        sum += wave_sum_u64(lane <= nearest ? (w & ST_VAL) : 0);
        if (nearest < 64) break;
        top -= 64;
    }
    if (lane == 0) st_publish(&status[i], ST_PRE | (sum + count));
    return sum;
}


// Plain word copy (device to device) and strided key extraction.
__global__ void k_copy_words(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
__global__ void k_extract_keys(const uint64_t* __restrict__ rows, uint64_t n, uint32_t stride,
                               uint64_t* __restrict__ keys) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        keys[i] = rows[i * stride];
}

// Stratified key sample: key of row floor((2q+1) n / 2S) for q < S.
__global__ void k_sample_keys(ColView src, uint64_t n, uint64_t S, uint64_t* __restrict__ out) {
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < S; q += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t pos = stratum_row(q, n, S);
        out[q] = src.key[pos * src.stride];
    }
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ---------------------------------------------------------------------------
// Single-key leaves: every row has the same key; reduce in pieces, then
// combine the pieces' partials with a fixed tree.
// ---------------------------------------------------------------------------

template <int NT>
__device__ __forceinline__ void block_reduce_agg(Agg& a, Agg* s_agg) {
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

// ---------------------------------------------------------------------------
// Leaf sort-reduce with direct placement: one workgroup per key range.  Leaves
// are taken in ticket order, which is their key order within each
// destination; a leaf's groups go straight to its destination at the chained
// prefix of the group counts of the destination's earlier leaves.
// Kind 0: at most LEAF_CAP rows, loaded, sorted in LDS (ordered on their top
// LEAF_SORT_BITS bits relative to the leaf minimum; runs of distinct keys that
// share those bits are then ordered by rank, or, if such runs are long or
// many, the leaf is re-sorted on all bits) and reduced.  Kind 1: a single key, whose
// pieces were reduced by k_single_partial; combined here with a fixed tree.
// ---------------------------------------------------------------------------

// Output rows of a leaf are staged in the sort area once the sort is done and
// leave in contiguous stores (a lane per 8-byte word), so that one store
// instruction writes whole cache lines instead of one row per lane.
constexpr int LEAF_STAGE_WORDS = (int)(sizeof(CSortSmem<LEAF_NT, LEAF_IPT>) / 8);

struct LeafSmem {
    union alignas(16) {
        CSortSmem<LEAF_NT, LEAF_IPT> sort;
        uint64_t stage[LEAF_STAGE_WORDS];
    };
    uint64_t mm[2 * LEAF_NT / 64];
    Agg seg_w[LEAF_NT / 64];  // the segmented scan's wave partials
    uint32_t seg_wf[LEAF_NT / 64];
    uint32_t fix_runs[1 + 2 * 32];  // the clash fix-up's runs (count, then lo/hi pairs)
    uint32_t scan_tmp[LEAF_NT / 64 + 1];
};

constexpr int LEAF_ROUND = 8;  // payload loads issued together

__device__ __forceinline__ uint64_t dest_base(const Dest& D) { return D.base ? *D.base : 0ull; }
// The destination's columns as the leaves index them (by output row); a
// launch-local key column is shifted back by the base row.
__device__ __forceinline__ OutView dest_out(const Dest& D) {
    OutView o = D.out;
    if (D.key_local && o.key) o.key -= dest_base(D) * o.stride;
    return o;
}

// Words of one output row and whether the destination is row-major with the
// fields in state order right after the key (then a leaf's rows form one
// contiguous span).
__device__ __forceinline__ int out_words(const OutView& o, bool& row_major) {
    int w = 1;
    bool rm = true;
    auto at = [&](const void* p) {
        if (!p) return;
        rm = rm && (const uint64_t*)p == (const uint64_t*)o.key + w;
        ++w;
    };
    at(o.cnt);
    at(o.sum);
    at(o.mn);
    at(o.mx);
    at(o.fs);
    row_major = rm && o.stride == (uint64_t)w;
    return w;
}

__device__ __forceinline__ void stage_agg(uint64_t* r, const OutView& o, const Agg& a) {
    int i = 0;
    r[i++] = a.key;
    if (o.cnt) r[i++] = a.cnt;
    if (o.sum) r[i++] = a.sum;
    if (o.mn) r[i++] = (uint64_t)a.mn;
    if (o.mx) r[i++] = (uint64_t)a.mx;
    if (o.fs) r[i++] = (uint64_t)__double_as_longlong(a.fs);
}

// Copy the first `rows` staged rows to destination rows pos0.. (all threads).
__device__ __forceinline__ void flush_stage(const uint64_t* st, uint32_t rows, int W, bool row_major,
                                           const OutView& o, uint64_t pos0) {
    const int tid = threadIdx.x;
    if (row_major) {
        uint64_t* dst = o.key + pos0 * (uint64_t)W;
        const uint32_t nw = rows * (uint32_t)W;
        for (uint32_t i = tid; i < nw; i += blockDim.x) dst[i] = st[i];
        return;
    }
    int f = 0;
    auto col = [&](void* p) {
        if (!p && f > 0) return;
        uint64_t* c = (uint64_t*)p;
        for (uint32_t g = tid; g < rows; g += blockDim.x) c[(pos0 + g) * o.stride] = st[(uint64_t)g * W + f];
        ++f;
    };
    col(o.key);
    col(o.cnt);
    col(o.sum);
    col(o.mn);
    col(o.mx);
    col(o.fs);
}

// Sort, reduce and place one leaf of at most LEAF_CAP rows (workgroup-wide),
// with IPTC sorted positions per thread (IPTC * LEAF_NT >= n).
// li is the leaf's ticket, [first, last] the tickets of its destination d.
template <int IPTC>
__device__ __forceinline__ void leaf_sort_reduce_t(const ColView& V, const uint32_t n, const Dest& D,
                                                   const uint32_t li, const uint32_t first, const uint32_t last,
                                                   const uint32_t d, uint64_t* __restrict__ status,
                                                   uint64_t* __restrict__ totals, uint32_t* __restrict__ ctl,
                                                   LeafSmem& s, uint64_t& s_pre) {
    constexpr int NT = LEAF_NT, IPT = LEAF_IPT;
    constexpr int ipt = IPTC;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint64_t k[IPT];
    uint16_t v[IPT];
    uint64_t mn = ~0ull, mx = 0ull;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        // coalesced loads, moved to blocked order before sorting
        const uint32_t q = (uint32_t)(w * 64 * IPT + j * 64 + lane);
        v[j] = (uint16_t)q;
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
        k[j] = q < n ? k[j] - mn : range;  // padding sorts last
    }
    const int nbits = bit_length(range);
    const int lo_bit = nbits > LEAF_SORT_BITS ? nbits - LEAF_SORT_BITS : 0;
    // only the slots of the leaf's rows (and their padding) take part
    striped_to_blocked<NT, IPT, IPTC>(k, v, s.sort);
    block_sort_cnt<NT, IPT, IPTC>(k, v, lo_bit, nbits, s.sort);
    if (lo_bit > 0) {
        // Distinct keys that share the sorted top bits (a clash) are still in
        // input order.  Each run of equal top bits around a clash (found by
        // binary search: the top bits are sorted) is put in order by the
        // whole workgroup: every row's rank in the run is its count of
        // smaller keys plus equal keys before it.  More than LEAF_FIX_RUNS
        // clashes, or a run longer than LEAF_FIX_MAX rows, sends the leaf
        // through a full-width sort instead.
        auto top = [&](uint32_t p) { return s.sort.key[pad16((int)p)] >> lo_bit; };
        uint32_t cl = 0;  // bit j: positions p-1 and p clash (p = tid*ipt + j)
#pragma unroll
        for (int j = 0; j < ipt; ++j) {
            const int p = tid * ipt + j;
            if (p > 0 && p < (int)n) {
                const uint64_t a = s.sort.key[pad16(p - 1)], b = s.sort.key[pad16(p)];
                if (a != b && (a >> lo_bit) == (b >> lo_bit)) cl |= 1u << j;
            }
        }
        uint32_t* runs = s.fix_runs;  // [0]: clashes seen, then (lo, hi) per clash
        if (tid == 0) runs[0] = 0;
        if (__syncthreads_or(cl != 0)) {
            for (int j = 0; j < ipt; ++j) {
                if (!(cl & (1u << j))) continue;
                const uint32_t p = (uint32_t)(tid * ipt + j);
                const uint64_t t = top(p);
                uint32_t a = 0, b = p;
                while (a < b) {
                    const uint32_t m = (a + b) >> 1;
                    if (top(m) < t) a = m + 1;
                    else b = m;
                }
                const uint32_t lo = a;
                a = p;
                b = n;
                while (a < b) {
                    const uint32_t m = (a + b) >> 1;
                    if (top(m) <= t) a = m + 1;
                    else b = m;
                }
                const uint32_t slot = atomicAdd(&runs[0], 1u);
                if (slot < (uint32_t)LEAF_FIX_RUNS) {
                    runs[1 + 2 * slot] = lo;
                    runs[2 + 2 * slot] = a;
                }
            }
            __syncthreads();
            const uint32_t nc = runs[0];
            bool redo = nc > (uint32_t)LEAF_FIX_RUNS;
            for (uint32_t r = 0; r < nc && !redo; ++r) redo = runs[2 + 2 * r] - runs[1 + 2 * r] > (uint32_t)LEAF_FIX_MAX;
            if (redo) {
#pragma unroll
                for (int j = 0; j < IPT; ++j) {
                    if (j < ipt) {
                        k[j] = s.sort.key[pad16(tid * ipt + j)];
                        v[j] = s.sort.val[pad16(tid * ipt + j)];
                    }
                }
                __syncthreads();
                block_sort_cnt<NT, IPT, IPTC>(k, v, 0, nbits, s.sort);
            } else {
                // the counter area holds a run's rows in rank order
                static_assert(sizeof(s.sort.cnt) >= (size_t)LEAF_FIX_MAX * (sizeof(uint64_t) + sizeof(uint16_t)),
                              "the clash fix-up stages a run in the counter area");
                uint64_t* tk = reinterpret_cast<uint64_t*>(s.sort.cnt);
                uint16_t* tv = reinterpret_cast<uint16_t*>(tk + LEAF_FIX_MAX);
                for (uint32_t r = 0; r < nc; ++r) {
                    const uint32_t lo = runs[1 + 2 * r], hi = runs[2 + 2 * r];
                    bool seen = false;  // clashes of one run name it once each
                    for (uint32_t q = 0; q < r; ++q) seen |= runs[1 + 2 * q] == lo;
                    if (seen) continue;
                    const uint32_t L = hi - lo;
                    for (uint32_t i = tid; i < L; i += NT) {
                        const uint64_t kx = s.sort.key[pad16((int)(lo + i))];
                        uint32_t rank = 0;
                        for (uint32_t q = 0; q < L; ++q) {
                            const uint64_t kq = s.sort.key[pad16((int)(lo + q))];
                            rank += (kq < kx || (kq == kx && q < i)) ? 1u : 0u;
                        }
                        tk[rank] = kx;
                        tv[rank] = s.sort.val[pad16((int)(lo + i))];
                    }
                    __syncthreads();
                    for (uint32_t i = tid; i < L; i += NT) {
                        s.sort.key[pad16((int)(lo + i))] = tk[i];
                        s.sort.val[pad16((int)(lo + i))] = tv[i];
                    }
                    __syncthreads();
                }
            }
        }
    }

    // Blocked arrangement: thread t owns sorted positions [t*ipt, t*ipt+ipt).
    const int p0 = tid * ipt;
    uint64_t kk[IPT];
    uint16_t rw[IPT];
    uint32_t heads = 0;  // bit j: position p0+j starts a group
    int nrows = 0;
    uint64_t key_before = 0;  // the key (less the minimum) of position p0 - 1
    {
        uint64_t prev = p0 > 0 ? s.sort.key[pad16(p0 - 1)] : 0;
        key_before = prev;
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int p = p0 + j;
            if (j >= ipt) break;
            kk[j] = s.sort.key[pad16(p)];
            rw[j] = s.sort.val[pad16(p)];
            if (p < (int)n) {
                ++nrows;
                if (p == 0 || kk[j] != prev) heads |= 1u << j;
            }
            prev = kk[j];
        }
    }
    const uint32_t nheads = __popc(heads);
    uint32_t total;
    const uint32_t obase = block_exclusive_scan<NT>(nheads, s.scan_tmp, total);
    if (w == 0) {
        const uint64_t pre = chained_prefix(status, li, first, total, &ctl[1]);
        if (lane == 0) s_pre = pre + dest_base(D);
    }
    __syncthreads();
    // the sort area is free from here on (the scan above synchronised)
    bool row_major;
    const int W = out_words(D.out, row_major);
    const uint32_t stage_rows = (uint32_t)LEAF_STAGE_WORDS / (uint32_t)W;
    const uint64_t pre0 = s_pre;
    auto put = [&](uint32_t g, const Agg& a) {
        if (g < stage_rows) {
            stage_agg(s.stage + (uint64_t)g * W, D.out, a);
        } else {
            const uint64_t pos = pre0 + g;
            if (pos < D.capacity) store_agg(dest_out(D), pos, a);
        }
    };

    Agg acc, pre_a;  // the thread's open group; its rows before its first head
    empty_agg(acc);
    empty_agg(pre_a);
    bool have_head = false;
    uint32_t h = 0;
#pragma unroll
    for (int r0 = 0; r0 < ipt; r0 += LEAF_ROUND) {
        Agg pay[LEAF_ROUND];
#pragma unroll
        for (int j = 0; j < LEAF_ROUND; ++j)
            if (r0 + j < nrows) load_payload(V, rw[r0 + j], pay[j]);
#pragma unroll
        for (int j = 0; j < LEAF_ROUND; ++j) {
            if (r0 + j >= nrows) break;
            Agg& r = pay[j];
            r.key = kk[r0 + j] + mn;
            if (heads & (1u << (r0 + j))) {
                if (!have_head) {
                    pre_a = acc;
                    have_head = true;
                } else {
                    put(obase + h - 1, acc);
                }
                acc = r;
                ++h;
            } else {
                combine(acc, r);
            }
        }
    }
    // Groups that span threads: a segmented scan over the threads' open
    // groups (a thread with a head starts a segment).  The group open at the
    // end of the thread before ends with this thread's rows before its first
    // head: this thread places it, as group obase - 1; the last thread with
    // rows places the leaf's last group.
    Agg before, incl;
    seg_scan_agg<NT>(acc, have_head, before, incl, s.seg_w, s.seg_wf);
    if (have_head && tid > 0) {
        combine(before, pre_a);
        before.key = key_before + mn;
        put(obase - 1, before);
    }
    if (nrows > 0 && (uint32_t)tid == (n - 1) / (uint32_t)ipt) {
        incl.key = have_head ? acc.key : key_before + mn;
        put(total - 1, incl);
    }
    __syncthreads();
    const uint32_t staged = total < stage_rows ? total : stage_rows;
    const uint64_t room = D.capacity > pre0 ? D.capacity - pre0 : 0;
    flush_stage(s.stage, (uint64_t)staged < room ? staged : (uint32_t)room, W, row_major, dest_out(D), pre0);
    if (tid == 0 && li == last) totals[d] = pre0 + total;
}

// A leaf of n <= LEAF_CAP rows: the sort's positions per thread rounded up to
// 4, 8 or 16.
__device__ __forceinline__ void leaf_sort_reduce(const ColView& V, const uint32_t n, const Dest& D, const uint32_t li,
                                                 const uint32_t first, const uint32_t last, const uint32_t d,
                                                 uint64_t* __restrict__ status, uint64_t* __restrict__ totals,
                                                 uint32_t* __restrict__ ctl, LeafSmem& s, uint64_t& s_pre) {
    if (n <= 4u * LEAF_NT)
        leaf_sort_reduce_t<4>(V, n, D, li, first, last, d, status, totals, ctl, s, s_pre);
    else if (n <= 8u * LEAF_NT)
        leaf_sort_reduce_t<8>(V, n, D, li, first, last, d, status, totals, ctl, s, s_pre);
    else
        leaf_sort_reduce_t<LEAF_IPT>(V, n, D, li, first, last, d, status, totals, ctl, s, s_pre);
}

// Reduce all rows of a single-key range of any size in one workgroup
// (fixed per-thread order, then a fixed tree) and place its one group.
__device__ __forceinline__ void leaf_single_stream(const ColView& V, const uint64_t n, const Dest& D,
                                                   const uint32_t li, const uint32_t first, const uint32_t last,
                                                   const uint32_t d, uint64_t* __restrict__ status,
                                                   uint64_t* __restrict__ totals, uint32_t* __restrict__ ctl,
                                                   LeafSmem& s, uint64_t& s_pre) {
    constexpr int NT = LEAF_NT;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (w == 0) {
        const uint64_t pre = chained_prefix(status, li, first, 1, &ctl[1]);
        if (lane == 0) s_pre = pre + dest_base(D);
    }
    Agg a;
    empty_agg(a);
    for (uint64_t i = tid; i < n; i += NT) {
        Agg r;
        load_payload(V, i, r);
        combine(a, r);
    }
    Agg* red = reinterpret_cast<Agg*>(s.sort.key);
    block_reduce_agg<NT>(a, red);
    if (tid == 0) {
        a.key = V.key[0];
        const uint64_t pos = s_pre;
        if (pos < D.capacity) store_agg(dest_out(D), pos, a);
        if (li == last) totals[d] = pos + 1;
    }
}

__global__ void __launch_bounds__(LEAF_NT, 3) k_leaf(const Leaf* __restrict__ leaves,
                                                  const uint32_t* __restrict__ leaf_dest,
                                                  const uint32_t* __restrict__ first_seg,
                                                  const Dest* __restrict__ dests, const Agg* __restrict__ partials,
                                                  uint64_t* __restrict__ status, uint64_t* __restrict__ totals,
                                                  uint32_t* __restrict__ ctl) {
    constexpr int NT = LEAF_NT, IPT = LEAF_IPT;
    __shared__ LeafSmem s;
    __shared__ uint32_t s_li;
    __shared__ uint64_t s_pre;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_li = atomicAdd(&ctl[0], 1u);
    __syncthreads();
    const uint32_t li = s_li;
    const Leaf Lf = leaves[li];
    const uint32_t d = leaf_dest[li];
    const Dest D = dests[d];
    const uint32_t first = first_seg[d], last = first_seg[d + 1] - 1;

    if (Lf.kind == 1) {
        if (w == 0) {
            const uint64_t pre = chained_prefix(status, li, first, 1, &ctl[1]);
            if (lane == 0) s_pre = pre + dest_base(D);
        }
        Agg a;
        empty_agg(a);
        for (uint32_t i = tid; i < Lf.single_count; i += NT) combine(a, partials[Lf.single_first + i]);
        Agg* red = reinterpret_cast<Agg*>(s.sort.key);  // NT*48 bytes fit the key array
        block_reduce_agg<NT>(a, red);
        if (tid == 0) {
            a.key = partials[Lf.single_first].key;
            const uint64_t pos = s_pre;
            if (pos < D.capacity) store_agg(dest_out(D), pos, a);
            if (li == last) totals[d] = pos + 1;
        }
        return;
    }

    leaf_sort_reduce(Lf.src, (uint32_t)Lf.n, D, li, first, last, d, status, totals, ctl, s, s_pre);
}

// ---------------------------------------------------------------------------
// Flat plan: one partition level whose buckets are the leaves.  Every slot
// finds its rows from the scanned histogram on the device, so the whole plan
// runs without the host (and can be captured as one graph).  A bucket larger
// than a leaf that holds more than one key cannot be taken here: it raises
// bit 1 of the error word and the host redoes the call on the general path.
// ---------------------------------------------------------------------------

__device__ __forceinline__ ColView aos_view_d(const uint64_t* base, const Layout& L) {
    ColView v;
    v.key = base;
    v.cnt = L.cnt >= 0 ? base + L.cnt : nullptr;
    v.sum = L.sum >= 0 ? (const int64_t*)(base + L.sum) : nullptr;
    v.mn = L.mn >= 0 ? (const int64_t*)(base + L.mn) : nullptr;
    v.mx = L.mx >= 0 ? (const int64_t*)(base + L.mx) : nullptr;
    v.fs = L.fs >= 0 ? (const double*)(base + L.fs) : nullptr;
    v.stride = (uint64_t)L.words;
    return v;
}

// Pieces of the single-key buckets of one flat region whose single-key
// buckets are known in advance (their splitter ranges hold one key): block
// (s, p) reduces rows [p*SINGLE_CHUNK, (p+1)*SINGLE_CHUNK) of the s-th such
// bucket into partials[s*max_pieces + p]; pieces past the bucket's end exit.
__global__ void __launch_bounds__(256) k_flat_single_partial(const Region* __restrict__ regions,
                                                             const uint64_t* __restrict__ offs,
                                                             const uint64_t* __restrict__ part, Layout L,
                                                             const uint32_t* __restrict__ single_buckets,
                                                             uint32_t max_pieces, Agg* __restrict__ partials) {
    __shared__ Agg s_agg[256];
    const uint32_t si = blockIdx.x / max_pieces, p = blockIdx.x - si * max_pieces;
    const Region R = regions[0];
    const uint32_t b = single_buckets[si];
    const uint64_t rb = offs[R.hist_base];
    const uint64_t start = offs[R.hist_base + (uint64_t)b * R.n_chunks] - rb;
    const uint64_t end = b + 1 < R.nb ? offs[R.hist_base + (uint64_t)(b + 1) * R.n_chunks] - rb : R.n;
    const uint64_t p0 = (uint64_t)p * SINGLE_CHUNK;
    if (start + p0 >= end) return;
    const uint32_t n = (uint32_t)(end - start - p0 < SINGLE_CHUNK ? end - start - p0 : SINGLE_CHUNK);
    const ColView V = aos_view_d(part + (R.out_pos + start + p0) * (uint64_t)L.words, L);
    Agg a;
    empty_agg(a);
    for (uint32_t i = threadIdx.x; i < n; i += 256) {
        Agg r;
        load_payload(V, i, r);
        combine(a, r);
    }
    block_reduce_agg<256>(a, s_agg);
    if (threadIdx.x == 0) {
        a.key = V.key[0];
        partials[(uint64_t)si * max_pieces + p] = a;
    }
}

__device__ __forceinline__ void leaf_flat_slot(const FlatSlot* __restrict__ slots, const FlatInst* __restrict__ insts,
                                               const Region* __restrict__ regions,
                                               const uint64_t* __restrict__ splitters,
                                               const uint64_t* __restrict__ offs, const uint64_t* __restrict__ part,
                                               Layout L, const uint32_t* __restrict__ first_slot,
                                               const Dest* __restrict__ dests, uint64_t* __restrict__ status,
                                               uint64_t* __restrict__ totals, uint32_t* __restrict__ ctl,
                                               const uint32_t* __restrict__ single_of,
                                               const Agg* __restrict__ partials, uint32_t max_pieces, LeafSmem& s,
                                               uint32_t& s_li, uint64_t& s_pre) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_li = atomicAdd(&ctl[0], 1u);
    __syncthreads();
    const uint32_t li = s_li;
    const FlatSlot sl = slots[li];
    const uint32_t d = sl.dest;
    const Dest D = dests[d];
    const uint32_t first = first_slot[d], last = first_slot[d + 1] - 1;
    ColView V;
    uint64_t n;
    bool single = false;
    if (sl.kind == 0) {
        V = insts[sl.idx].src;
        n = insts[sl.idx].n;
    } else {
        const Region R = regions[sl.idx];
        const uint32_t b = sl.bucket;
        const uint64_t rb = offs[R.hist_base];
        const uint64_t start = offs[R.hist_base + (uint64_t)b * R.n_chunks] - rb;
        const uint64_t end = b + 1 < R.nb ? offs[R.hist_base + (uint64_t)(b + 1) * R.n_chunks] - rb : R.n;
        n = end - start;
        V = aos_view_d(part + (R.out_pos + start) * (uint64_t)L.words, L);
        const uint64_t* spl = splitters + (uint64_t)sl.idx * (MAX_BUCKETS - 1);
        const uint64_t lo = b ? spl[b - 1] : 0ull;
        const uint64_t hi = b + 1 < R.nb ? spl[b] - 1 : ~0ull;
        single = n > 0 && lo == hi;
    }
    if (n == 0 || (n > (uint64_t)LEAF_CAP && !single)) {
        if (n > 0 && tid == 0) {
            atomicOr(&ctl[1], 2u);
            __threadfence();  // the error bit is visible before this slot's prefix
        }
        if (w == 0) {
            const uint64_t pre = chained_prefix(status, li, first, 0, &ctl[1]);
            if (lane == 0 && li == last) totals[d] = pre + dest_base(D);
        }
        return;
    }
    if (single && single_of && single_of[sl.bucket] != ~0u) {
        // a single-key bucket whose pieces k_flat_single_partial reduced:
        // combine them with a fixed tree
        if (w == 0) {
            const uint64_t pre = chained_prefix(status, li, first, 1, &ctl[1]);
            if (lane == 0) s_pre = pre + dest_base(D);
        }
        const Agg* pa = partials + (uint64_t)single_of[sl.bucket] * max_pieces;
        const uint32_t np = (uint32_t)((n + SINGLE_CHUNK - 1) / SINGLE_CHUNK);
        Agg a;
        empty_agg(a);
        for (uint32_t i = tid; i < np; i += LEAF_NT) combine(a, pa[i]);
        Agg* red = reinterpret_cast<Agg*>(s.sort.key);  // LEAF_NT*48 bytes fit the key array
        block_reduce_agg<LEAF_NT>(a, red);
        if (tid == 0) {
            a.key = pa[0].key;
            if (s_pre < D.capacity) store_agg(dest_out(D), s_pre, a);
            if (li == last) totals[d] = s_pre + 1;
        }
        return;
    }
    if (single) leaf_single_stream(V, n, D, li, first, last, d, status, totals, ctl, s, s_pre);
    else leaf_sort_reduce(V, (uint32_t)n, D, li, first, last, d, status, totals, ctl, s, s_pre);
}

// host_out (optional): a device-mapped pinned slot.  The last slot hands
// the control word (ticket, error bits) and destination 0's end row to the
// host there, so that no copy needs to follow the launch.
__global__ void __launch_bounds__(LEAF_NT, 3) k_leaf_flat(const FlatSlot* __restrict__ slots,
                                                       const FlatInst* __restrict__ insts,
                                                       const Region* __restrict__ regions,
                                                       const uint64_t* __restrict__ splitters,
                                                       const uint64_t* __restrict__ offs,
                                                       const uint64_t* __restrict__ part, Layout L,
                                                       const uint32_t* __restrict__ first_slot,
                                                       const Dest* __restrict__ dests, uint64_t* __restrict__ status,
                                                       uint64_t* __restrict__ totals, uint32_t* __restrict__ ctl,
                                                       const uint32_t* __restrict__ single_of,
                                                       const Agg* __restrict__ partials, uint32_t max_pieces,
                                                       uint64_t* __restrict__ host_out) {
    __shared__ LeafSmem s;
    __shared__ uint32_t s_li;
    __shared__ uint64_t s_pre;
    leaf_flat_slot(slots, insts, regions, splitters, offs, part, L, first_slot, dests, status, totals, ctl, single_of,
                   partials, max_pieces, s, s_li, s_pre);
    if (host_out && threadIdx.x == 0 && s_li + 1 == gridDim.x) {
        __threadfence();
        host_out[1] = totals[0];
        host_out[0] = __hip_atomic_load(reinterpret_cast<uint64_t*>(ctl), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// LDS-staged merge of two sorted runs of unique keys, both row-major with
// the same layout, combining equal keys (A's row first).  Partition p covers
// merge diagonals [p*MG_D, (p+1)*MG_D); its A and B rows are copied to LDS
// with coalesced loads and merged there by merge path per thread.  Each
// thread holds its merged rows in registers, writes them back over the LDS
// input at their merged position, and the partition's output leaves in
// contiguous stores at the chained prefix of the partitions' group counts.
// ---------------------------------------------------------------------------

// Copies na words of a and then nb words of b to dst[0, na + nb) in LDS,
// NT threads with LOADS loads in flight each.  (A loop of one load and one
// LDS store per trip waits for each load before the next is issued: one
// memory latency per trip.)
template <int NT, int LOADS>
__device__ __forceinline__ void stage_words(uint64_t* dst, const uint64_t* __restrict__ a, uint32_t na,
                                            const uint64_t* __restrict__ b, uint32_t nb) {
    const uint32_t n = na + nb;
    for (uint32_t base = threadIdx.x; base < n; base += NT * LOADS) {
        uint64_t r[LOADS];
#pragma unroll
        for (int q = 0; q < LOADS; ++q) {
            const uint32_t x = base + (uint32_t)q * NT;
            if (x < n) r[q] = x < na ? a[x] : b[x - na];
        }
#pragma unroll
        for (int q = 0; q < LOADS; ++q) {
            const uint32_t x = base + (uint32_t)q * NT;
            if (x < n) dst[x] = r[q];
        }
    }
}

constexpr int MG_NT = 512;
constexpr int MG_PER = 2;
constexpr int MG_D = MG_NT * MG_PER;
constexpr int MG_MAXW = 6;
constexpr uint64_t MG_GRID = 256;

// Split of diagonal d over row-major key columns (stride w words); an equal
// pair is never separated (its B row goes with the A row before the split).
__device__ __forceinline__ void merge_split_rows(const uint64_t* A, uint64_t na, const uint64_t* B, uint64_t nb,
                                                 uint32_t w, uint64_t d, uint64_t& i_out, uint64_t& j_out) {
    uint64_t lo = d > nb ? d - nb : 0;
    uint64_t hi = d < na ? d : na;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (A[mid * w] <= B[(d - 1 - mid) * w]) lo = mid + 1;
        else hi = mid;
    }
    uint64_t i = lo, j = d - lo;
    if (i > 0 && j < nb && A[(i - 1) * w] == B[j * w]) ++j;
    i_out = i;
    j_out = j;
}

// One thread per partition boundary: splits[2*p], splits[2*p+1].
__global__ void k_merge_splits(const uint64_t* __restrict__ A, uint64_t na, const uint64_t* __restrict__ B,
                               uint64_t nb, uint32_t w, uint64_t parts, uint64_t* __restrict__ splits) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > parts) return;
    uint64_t d = p * MG_D;
    if (d > na + nb) d = na + nb;
    uint64_t i, j;
    merge_split_rows(A, na, B, nb, w, d, i, j);
    splits[2 * p] = i;
    splits[2 * p + 1] = j;
}

__device__ __forceinline__ void combine_rows(uint64_t* o, const uint64_t* a, const uint64_t* b, const Layout& L) {
    o[0] = a[0];
    if (L.cnt >= 0) o[L.cnt] = a[L.cnt] + b[L.cnt];
    if (L.sum >= 0) o[L.sum] = a[L.sum] + b[L.sum];
    if (L.mn >= 0) o[L.mn] = (uint64_t)((int64_t)a[L.mn] < (int64_t)b[L.mn] ? (int64_t)a[L.mn] : (int64_t)b[L.mn]);
    if (L.mx >= 0) o[L.mx] = (uint64_t)((int64_t)a[L.mx] > (int64_t)b[L.mx] ? (int64_t)a[L.mx] : (int64_t)b[L.mx]);
    if (L.fs >= 0) o[L.fs] = __double_as_longlong(__longlong_as_double(a[L.fs]) + __longlong_as_double(b[L.fs]));
}

// next_ctl (optional, next_words words): the control block of the next merge
// on the stream, cleared here so that it needs no launch of its own.
//
// In place.  A may lie in the output buffer itself: partitions are taken in
// ticket order, and a partition stages all its input in LDS before it
// publishes its count, so when a partition writes, every partition of an
// earlier ticket has read its input.
//  - Forward (rev_cap == 0): out is written from its start; A may occupy the
//    tail of a buffer of at least na + nb rows ending where A ends.  A write
//    of partition p ends before diagonal d_{p+1} <= ia_{p+1} + nb, which is
//    not beyond where the A rows of later partitions start.
//  - Reverse (rev_cap = C > 0): partitions are taken from the last key down
//    and the merged rows end at row C of out (C >= na + nb); A may occupy
//    rows [0, na) of out.  A write of partition p starts at or after
//    C - (na - ia_p) - (nb - ja_p) >= ia_p, beyond the A rows of every
//    partition taken later.
__global__ void __launch_bounds__(MG_NT) k_merge(const uint64_t* A, uint64_t na,
                                                 const uint64_t* __restrict__ B, uint64_t nb,
                                                 const uint64_t* __restrict__ splits, uint64_t* out,
                                                 Layout L, uint64_t* __restrict__ status, uint32_t* __restrict__ ctl,
                                                 uint64_t* __restrict__ total_out, uint64_t* __restrict__ next_ctl,
                                                 uint32_t next_words, uint32_t nparts,
                                                 uint64_t* __restrict__ host_out, uint64_t rev_cap) {
    __shared__ uint64_t s_in[(MG_D + 2) * MG_MAXW];
    __shared__ uint32_t s_li[MG_NT + 1], s_lj[MG_NT + 1];
    __shared__ uint32_t s_tmp[MG_NT / 64 + 1];
    __shared__ uint32_t s_part;
    __shared__ uint64_t s_pre;
    const int tid = threadIdx.x;
    const uint32_t W = (uint32_t)L.words;
    for (uint32_t x = blockIdx.x * MG_NT + tid; x < next_words; x += gridDim.x * MG_NT) next_ctl[x] = 0;
    // a persistent grid: each workgroup takes partitions in ticket order
    for (;;) {
        if (tid == 0) s_part = atomicAdd(&ctl[0], 1u);
        __syncthreads();
        const uint32_t ticket = s_part;
        if (ticket >= nparts) break;
        const uint32_t part = rev_cap ? nparts - 1 - ticket : ticket;
        const uint64_t ia0 = splits[2 * part], ja0 = splits[2 * part + 1];
        const uint64_t ia1 = splits[2 * part + 2], ja1 = splits[2 * part + 3];
        const uint32_t la = (uint32_t)(ia1 - ia0), lb = (uint32_t)(ja1 - ja0);
        // a partition is about MG_D rows: 12 words per thread in one round
        stage_words<MG_NT, 12>(s_in, A + ia0 * W, la * W, B + ja0 * W, lb * W);
        __syncthreads();
        const uint64_t* a = s_in;
        const uint64_t* b = s_in + la * W;
        {
            // local split of this thread's diagonal
            uint32_t d = (uint32_t)tid * MG_PER;
            if (d > la + lb) d = la + lb;
            uint32_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (a[mid * W] <= b[(d - 1 - mid) * W]) lo = mid + 1;
                else hi = mid;
            }
            uint32_t i = lo, j = d - lo;
            if (i > 0 && j < lb && a[(i - 1) * W] == b[j * W]) ++j;
            s_li[tid] = i;
            s_lj[tid] = j;
            if (tid == 0) {
                s_li[MG_NT] = la;
                s_lj[MG_NT] = lb;
            }
        }
        __syncthreads();
        const uint32_t i0 = s_li[tid], i1 = s_li[tid + 1] > i0 ? s_li[tid + 1] : i0;
        const uint32_t j0 = s_lj[tid], j1 = s_lj[tid + 1] > j0 ? s_lj[tid + 1] : j0;
        // a thread's inputs span at most MG_PER + 1 rows (its end split may
        // carry an equal pair's B row), so it makes at most MG_PER + 1 rows
        constexpr int RMAX = MG_PER + 1;
        uint64_t rows[RMAX][MG_MAXW];
        uint32_t c = 0;
        {
            uint32_t i = i0, j = j0;
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (i < i1 || j < j1) {
                    const uint64_t* src;
                    const uint64_t* src2 = nullptr;
                    if (j >= j1 || (i < i1 && a[i * W] < b[j * W])) {
                        src = a + i * W;
                        ++i;
                    } else if (i >= i1 || b[j * W] < a[i * W]) {
                        src = b + j * W;
                        ++j;
                    } else {
                        src = a + i * W;
                        src2 = b + j * W;
                        ++i;
                        ++j;
                    }
#pragma unroll
                    for (int x = 0; x < MG_MAXW; ++x) rows[r][x] = x < (int)W ? src[x] : 0;
                    if (src2) {
                        uint64_t t[MG_MAXW];
                        combine_rows(t, src, src2, L);
#pragma unroll
                        for (int x = 0; x < MG_MAXW; ++x)
                            if (x < (int)W) rows[r][x] = t[x];
                    }
                    ++c;
                }
            }
        }
        uint32_t tot;
        const uint32_t off = block_exclusive_scan<MG_NT>(c, s_tmp, tot);  // synchronises: the input is dead
        if (tid < 64) {
            const uint64_t pre = chained_prefix(status, ticket, 0, tot, &ctl[1]);
            if (tid == 0) {
                s_pre = pre;
                if (ticket == nparts - 1) {
                    *total_out = pre + tot;
                    if (host_out) {
                        __threadfence();
                        host_out[1] = pre + tot;
                        host_out[0] = __hip_atomic_load(reinterpret_cast<uint64_t*>(ctl), __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if ((uint32_t)r < c) {
#pragma unroll
                for (int x = 0; x < MG_MAXW; ++x)
                    if (x < (int)W) s_in[(off + r) * W + x] = rows[r][x];
            }
        }
        __syncthreads();
        uint64_t* const ob = out + (rev_cap ? rev_cap - s_pre - tot : s_pre) * W;
        for (uint32_t x = tid; x < tot * W; x += MG_NT) ob[x] = s_in[x];
        __syncthreads();  // the LDS input and s_part are reused by the next partition
    }
}

// ---------------------------------------------------------------------------
// Replacement selection through the index (Section 3): eviction scans the
// index in key order from a cursor.  cur[0] is the cursor key and cur[1] is 1
// once the scan has passed the largest key value.
// ---------------------------------------------------------------------------

// First row of the merged index U (*m rows, stride w words) whose key is at or
// after the cursor, by a 64-way search (one wave); m when the scan is past
// the end.
__global__ void __launch_bounds__(64) k_rs_probe(const uint64_t* __restrict__ U, const uint64_t* __restrict__ m_ptr,
                                                 uint32_t w, const uint64_t* __restrict__ cur,
                                                 uint64_t* __restrict__ p_out) {
    const int lane = threadIdx.x;
    const uint64_t m = *m_ptr, c = cur[0];
    uint64_t lo = 0, hi = cur[1] ? 0 : m;
    if (cur[1]) lo = m;
    while (lo < hi) {
        // probes lo + k*step (k < 64); keys below c form a prefix
        const uint64_t step = (hi - lo) / 65 + 1;
        const uint64_t q = lo + (uint64_t)lane * step;
        const bool in = q < hi;
        const bool below = in && U[q * w] < c;
        const uint64_t above = __ballot(in && !below);
        if (above) {
            const int f = __ffsll((long long)above) - 1;
            const uint64_t nlo = f > 0 ? lo + (uint64_t)(f - 1) * step + 1 : lo;
            hi = lo + (uint64_t)f * step;
            lo = nlo;
        } else {
            const uint64_t bm = __ballot(below);
            lo = lo + (uint64_t)(63 - __clzll((long long)bm)) * step + 1;
        }
    }
    if (lane == 0) *p_out = lo;
}

// Evict e = a + b rows of U (m rows): rows [p, p+a) end the open run and rows
// [0, b) start the next one.  The kept rows [b, p) and [p+a, m) go to out
// rows [0, m-e) in order; the evicted rows follow at out rows [m-e, m) in run
// order.  The cursor moves just past the last evicted key.
__global__ void __launch_bounds__(256) k_rs_evict(const uint64_t* __restrict__ U, uint64_t m, uint32_t w, uint64_t p,
                                                  uint64_t a, uint64_t b, uint64_t* __restrict__ out,
                                                  uint64_t* __restrict__ cur) {
    const uint64_t kept = m - a - b;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t o;
        if (i < b) o = kept + a + i;
        else if (i < p) o = i - b;
        else if (i < p + a) o = kept + (i - p);
        else o = i - a - b;
        const uint64_t* src = U + i * w;
        uint64_t* dst = out + o * w;
        for (uint32_t x = 0; x < w; ++x) dst[x] = src[x];
        const uint64_t last = b ? b - 1 : p + a - 1;
        if (i == last) {
            const uint64_t k = src[0];
            cur[0] = k + 1;
            cur[1] = k == ~0ull ? 1ull : 0ull;
        }
    }
}

// ---------------------------------------------------------------------------
// Sorted-input path: input already ordered on its key is grouped in one
// stream, with no sort (in-stream aggregation).  Nominal tiles of SORTED_T
// rows count their group heads (a row whose key differs from the row
// before); tile boundaries move forward to the next head, so that every range
// between moved boundaries holds whole groups.  One workgroup reduces a range;
// a group longer than a tile is reduced in parallel pieces.  Keys may be
// grouped on their high bits only (key >> shift).
// ---------------------------------------------------------------------------

constexpr uint32_t SORTED_T = 3584;                 // nominal tile rows
constexpr uint32_t SORTED_CAP = (uint32_t)LEAF_CAP;  // rows one workgroup reduces
constexpr int SORTED_NT = 256;

__device__ __forceinline__ uint64_t skey(const ColView& V, uint64_t i, int shift) { return V.key[i * V.stride] >> shift; }

// heads[t]: group heads in tile t; *bad = 1 if some key is below its predecessor.
__global__ void __launch_bounds__(SORTED_NT) k_sorted_tiles(ColView V, uint64_t n, int shift,
                                                            uint32_t* __restrict__ heads, uint32_t* __restrict__ bad) {
    __shared__ uint32_t s_tmp[SORTED_NT / 64 + 1];
    const uint64_t t0 = (uint64_t)blockIdx.x * SORTED_T;
    uint32_t c = 0;
    bool desc = false;
    for (uint32_t j = threadIdx.x; j < SORTED_T; j += SORTED_NT) {
        const uint64_t i = t0 + j;
        if (i >= n) break;
        const uint64_t k = skey(V, i, shift);
        if (i == 0) {
            ++c;
            continue;
        }
        const uint64_t q = skey(V, i - 1, shift);
        c += k != q ? 1u : 0u;
        desc |= k < q;
    }
    uint32_t tot;
    block_exclusive_scan<SORTED_NT>(c, s_tmp, tot);
    const bool any_desc = __syncthreads_or(desc);
    if (threadIdx.x == 0) {
        heads[blockIdx.x] = tot;
        if (any_desc) atomicOr(bad, 1u);
    }
}

// bounds[t] for t in [1, m): the first head at or after t*SORTED_T (or n);
// bounds[0] = 0 and bounds[m] = n.  Galloping search: a long group costs
// O(log length).
__global__ void k_sorted_align(ColView V, uint64_t n, int shift, uint64_t m, uint64_t* __restrict__ bounds) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > m) return;
    if (t == 0 || t == m) {
        bounds[t] = t == 0 ? 0 : n;
        return;
    }
    const uint64_t b = t * SORTED_T;
    const uint64_t x = skey(V, b - 1, shift);
    if (skey(V, b, shift) != x) {
        bounds[t] = b;
        return;
    }
    uint64_t lo = b, hi = n, step = 1;
    for (;;) {
        const uint64_t c = lo + step;
        if (c >= n) {
            hi = n;
            break;
        }
        if (skey(V, c, shift) != x) {
            hi = c;
            break;
        }
        lo = c;
        step <<= 1;
    }
    while (lo + 1 < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (skey(V, mid, shift) == x) lo = mid;
        else hi = mid;
    }
    bounds[t] = hi;
}

struct SortedSmem {
    uint64_t col[SORTED_CAP];  // one column of the range, for the striped-to-blocked transpose
    Agg seg_w[SORTED_NT / 64];  // the segmented scan's wave partials
    uint32_t seg_wf[SORTED_NT / 64];
    uint32_t tmp[SORTED_NT / 64 + 1];
};

constexpr int SORTED_IPT = (int)SORTED_CAP / SORTED_NT;

// Words of column c of rows [s, s+n) into x[] in blocked order (thread t holds
// rows t*ipt ..), through LDS with coalesced loads.
__device__ __forceinline__ void sorted_column(const uint64_t* c, uint64_t stride, uint64_t s, uint32_t n, int shift,
                                              uint32_t p0, uint32_t ipt, uint64_t (&x)[SORTED_IPT], SortedSmem& sm) {
#pragma unroll
    for (int j = 0; j < SORTED_IPT; ++j) {
        const uint32_t q = (uint32_t)j * SORTED_NT + threadIdx.x;
        if (q < n) sm.col[q] = c[(s + q) * stride] >> shift;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SORTED_IPT; ++j)
        if ((uint32_t)j < ipt && p0 + j < n) x[j] = sm.col[p0 + j];
    __syncthreads();
}

// Groups of rows [s, s+n) (n <= SORTED_CAP; row s starts a group) written at
// out[g ..).  Blocked: thread t reduces rows t*ipt .. t*ipt+ipt-1; the group
// open at a thread's end continues into the following threads.  Returns the
// number of groups.
__device__ uint32_t sorted_reduce_range(const ColView& V, int shift, uint64_t s, uint32_t n, const OutView& out,
                                        uint64_t cap, uint64_t g, SortedSmem& sm) {
    const int tid = threadIdx.x;
    const uint32_t ipt = (n + SORTED_NT - 1) / SORTED_NT;
    const uint32_t p0 = (uint32_t)tid * ipt;
    const uint32_t p1 = p0 + ipt < n ? p0 + ipt : n;
    uint64_t kk[SORTED_IPT], cc[SORTED_IPT], vv[SORTED_IPT], ff[SORTED_IPT];
    // keys, and the key before the thread's first row
#pragma unroll
    for (int j = 0; j < SORTED_IPT; ++j) {
        const uint32_t q = (uint32_t)j * SORTED_NT + tid;
        if (q < n) sm.col[q] = skey(V, s + q, shift);
    }
    __syncthreads();
    const uint64_t first_prev = p0 > 0 && p0 < n ? sm.col[p0 - 1] : 0;
#pragma unroll
    for (int j = 0; j < SORTED_IPT; ++j)
        if ((uint32_t)j < ipt && p0 + j < n) kk[j] = sm.col[p0 + j];
    __syncthreads();
    if (V.cnt) sorted_column(V.cnt, V.stride, s, n, 0, p0, ipt, cc, sm);
    if (V.sum) sorted_column((const uint64_t*)V.sum, V.stride, s, n, 0, p0, ipt, vv, sm);
    if (V.fs) sorted_column((const uint64_t*)V.fs, V.stride, s, n, 0, p0, ipt, ff, sm);
    uint32_t nh = 0;
    {
        uint64_t prev = first_prev;
#pragma unroll
        for (int j = 0; j < SORTED_IPT; ++j) {
            const uint32_t p = p0 + j;
            if (p < p1) {
                if (p == 0 || kk[j] != prev) ++nh;
                prev = kk[j];
            }
        }
    }
    uint32_t total;
    const uint32_t obase = block_exclusive_scan<SORTED_NT>(nh, sm.tmp, total);
    Agg acc, pre_a;  // the thread's open group; its rows before its first head
    empty_agg(acc);
    empty_agg(pre_a);
    bool have_head = false;
    uint32_t h = 0;
    uint64_t prev = first_prev;
#pragma unroll
    for (int j = 0; j < SORTED_IPT; ++j) {
        const uint32_t p = p0 + j;
        if (p >= p1) break;
        Agg r;
        r.key = kk[j];
        r.cnt = V.cnt ? cc[j] : 1ull;
        r.sum = V.sum ? vv[j] : 0ull;
        r.mn = V.sum ? (int64_t)vv[j] : INT64_MAX;
        r.mx = V.sum ? (int64_t)vv[j] : INT64_MIN;
        r.fs = V.fs ? __longlong_as_double((long long)ff[j]) : 0.0;
        if (p == 0 || r.key != prev) {
            if (!have_head) {
                pre_a = acc;
                have_head = true;
            } else {
                const uint64_t pos = g + obase + h - 1;
                if (pos < cap) store_agg(out, pos, acc);
            }
            acc = r;
            ++h;
        } else {
            combine(acc, r);
        }
        prev = r.key;
    }
    // groups that span threads: the segmented scan of the leaf kernels
    Agg before, incl;
    seg_scan_agg<SORTED_NT>(acc, have_head, before, incl, sm.seg_w, sm.seg_wf);
    if (have_head && tid > 0) {
        combine(before, pre_a);
        before.key = first_prev;
        const uint64_t pos = g + obase - 1;
        if (pos < cap) store_agg(out, pos, before);
    }
    if (p1 > p0 && (uint32_t)tid == (n - 1) / ipt) {
        incl.key = have_head ? acc.key : first_prev;
        const uint64_t pos = g + total - 1;
        if (pos < cap) store_agg(out, pos, incl);
    }
    return total;
}

// One workgroup per range [bounds[t], bounds[t+1]).  A range longer than
// SORTED_CAP ends with a group that crosses the next nominal boundary: its
// rows before that group (less than a tile) are reduced here and the group
// itself is listed in bigs (first row, end, output position) for the
// piecewise reduction.
__global__ void __launch_bounds__(SORTED_NT) k_sorted_ranges(ColView V, uint64_t n, int shift,
                                                             const uint64_t* __restrict__ bounds,
                                                             const uint64_t* __restrict__ offs, OutView out,
                                                             uint64_t cap, uint64_t* __restrict__ bigs,
                                                             uint32_t* __restrict__ n_bigs) {
    __shared__ SortedSmem sm;
    __shared__ uint32_t s_tmp2[SORTED_NT / 64 + 1];
    __shared__ uint64_t s_last;
    const uint64_t t = blockIdx.x;
    const uint64_t a = bounds[t], e = bounds[t + 1];
    if (a >= e) return;
    const int tid = threadIdx.x;
    // output position of the group starting at a: heads before a
    const uint64_t u = a / SORTED_T, bu = u * SORTED_T;
    uint32_t c = 0;
    for (uint64_t i = bu + tid; i < a; i += SORTED_NT)
        c += (i == 0 || skey(V, i, shift) != skey(V, i - 1, shift)) ? 1u : 0u;
    uint32_t before;
    block_exclusive_scan<SORTED_NT>(c, s_tmp2, before);
    const uint64_t g = offs[u] + before;
    if (e - a <= SORTED_CAP) {
        sorted_reduce_range(V, shift, a, (uint32_t)(e - a), out, cap, g, sm);
        return;
    }
    // the last head before the next nominal boundary starts the long group
    const uint64_t nb = (t + 1) * SORTED_T;
    if (tid == 0) s_last = a;
    __syncthreads();
    for (uint64_t i = a + 1 + tid; i < nb; i += SORTED_NT)
        if (skey(V, i, shift) != skey(V, i - 1, shift)) atomicMax((unsigned long long*)&s_last, (unsigned long long)i);
    __syncthreads();
    const uint64_t L = s_last;
    uint32_t small = 0;
    if (L > a) small = sorted_reduce_range(V, shift, a, (uint32_t)(L - a), out, cap, g, sm);
    if (tid == 0) {
        const uint32_t k = atomicAdd(n_bigs, 1u);
        bigs[3 * k] = L;
        bigs[3 * k + 1] = e;
        bigs[3 * k + 2] = g + small;
    }
}

// Long groups: combine the partials of each group's pieces (k_single_partial)
// with a fixed tree and write the group at its position.  big b owns partials
// [first[b], first[b+1]).
__global__ void __launch_bounds__(256) k_sorted_big_final(ColView V, int shift, const uint64_t* __restrict__ bigs,
                                                          const uint32_t* __restrict__ first,
                                                          const Agg* __restrict__ partials, OutView out,
                                                          uint64_t cap) {
    __shared__ Agg s_agg[256];
    const uint32_t b = blockIdx.x;
    Agg a;
    empty_agg(a);
    for (uint32_t i = first[b] + threadIdx.x; i < first[b + 1]; i += 256) combine(a, partials[i]);
    block_reduce_agg<256>(a, s_agg);
    if (threadIdx.x == 0) {
        a.key = skey(V, bigs[3 * b], shift);
        const uint64_t pos = bigs[3 * b + 2];
        if (pos < cap) store_agg(out, pos, a);
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

// Single workgroup exclusive scan of a short count array (at most a few tiles
// of SMALL_SCAN_TILE): one launch instead of three.
constexpr int SMALL_SCAN_NT = 1024;
constexpr int SMALL_SCAN_IPT = 16;
constexpr uint64_t SMALL_SCAN_TILE = (uint64_t)SMALL_SCAN_NT * SMALL_SCAN_IPT;
constexpr uint64_t SMALL_SCAN_MAX = 4 * SMALL_SCAN_TILE;

__global__ void __launch_bounds__(SMALL_SCAN_NT) k_scan_small(const uint32_t* __restrict__ in, uint64_t n,
                                                              uint64_t* __restrict__ out) {
    __shared__ uint32_t s_tmp[SMALL_SCAN_NT / 64 + 1];
    uint64_t carry = 0;
    for (uint64_t b0 = 0; b0 < n; b0 += SMALL_SCAN_TILE) {
        const uint64_t base = b0 + (uint64_t)threadIdx.x * SMALL_SCAN_IPT;
        uint32_t loc[SMALL_SCAN_IPT];
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < SMALL_SCAN_IPT; ++j) {
            loc[j] = base + j < n ? in[base + j] : 0u;
            acc += loc[j];
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<SMALL_SCAN_NT>(acc, s_tmp, tot);
        uint64_t run = carry + ex;
#pragma unroll
        for (int j = 0; j < SMALL_SCAN_IPT; ++j) {
            if (base + j < n) out[base + j] = run;
            run += loc[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
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

// Rows [*lo, *hi) of the output (below cap) from a launch-local key buffer:
// key i belongs to output row *lo + i.
__global__ void k_unpack_pairs_at(const uint64_t* __restrict__ keys, const uint64_t* __restrict__ lo,
                                  const uint64_t* __restrict__ hi, uint64_t cap, int32_t* __restrict__ a,
                                  int32_t* __restrict__ b) {
    const uint64_t r0 = lo ? *lo : 0ull, r1 = *hi < cap ? *hi : cap;
    const uint64_t n = r1 > r0 ? r1 - r0 : 0ull;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const uint64_t k = keys[i];
        a[r0 + i] = (int32_t)((uint32_t)(k >> 32) ^ 0x80000000u);
        b[r0 + i] = (int32_t)((uint32_t)k ^ 0x80000000u);
    }
}

// The int32 value held in the high half of a normalized pair key.
__global__ void k_unpack_hi(const uint64_t* __restrict__ hi, uint64_t n, int32_t* __restrict__ a) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        a[i] = (int32_t)((uint32_t)hi[i] ^ 0x80000000u);
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

// The chunk is read in rows of 256 consecutive elements, one per thread
// (coalesced, as in k_seg_count); a row holding segment starts places them
// in order by wave ballots and the waves' counts, and a row without any is
// skipped after one block-wide vote.  (A thread walking a contiguous
// sub-range of its own made every load of a wave touch a different line:
// 6.7 ms for 200M rows, against 0.4 ms for the count.)
__global__ void __launch_bounds__(256) k_seg_write(const int32_t* __restrict__ a, uint64_t n, uint32_t chunk,
                                                   const uint64_t* __restrict__ offs, uint64_t* __restrict__ starts) {
    __shared__ uint32_t s_w[256 / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t c0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    uint64_t o = offs[blockIdx.x];  // starts before this chunk
    for (uint64_t base = c0; base < c1; base += 256) {
        const uint64_t i = base + (uint64_t)tid;
        const bool f = i < c1 && (i == 0 || a[i] != a[i - 1]);
        if (!__syncthreads_or(f)) continue;
        const uint64_t bal = __ballot(f);
        if (lane == 0) s_w[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < 256 / 64; ++q) {
            before += q < w ? s_w[q] : 0u;
            tot += s_w[q];
        }
        if (f) starts[o + before + (uint64_t)__popcll(bal & ((1ull << lane) - 1ull))] = i;
        o += tot;
        __syncthreads();  // s_w is rewritten by the next row with starts
    }
}


// ---------------------------------------------------------------------------
// Compact run format.  A state row whose count is 1 holds a single input row,
// so key plus raw value columns describe it; a row whose count and integer
// aggregates fit in 32 bits is packed (packed_words).  A run is written as
// the sorted sub-run of count-1 rows, column by column (single_bytes), then
// the sorted sub-run of packed rows, then the sorted sub-run of the other
// rows in state layout (a stable three-way split, two passes).  The integer
// column of the count-1 part takes 4 bytes per value when every value in it
// fits in 32 bits.
// ---------------------------------------------------------------------------

constexpr int SPLIT_T = 4096;  // rows per workgroup

__device__ __forceinline__ bool fits_i32(uint64_t v) { return (int64_t)v == (int64_t)(int32_t)(int64_t)v; }

// A state row (count above 1) that the packed format holds exactly.
__device__ __forceinline__ bool packable(const uint64_t* q, const Layout& S) {
    if (!has_packed(S) || (q[S.cnt] >> 32) != 0) return false;
    return S.sum < 0 || (fits_i32(q[S.sum]) && fits_i32(q[S.mn]) && fits_i32(q[S.mx]));
}

// counts[b]: count-1 rows of block b, counts[nblk + b]: its packed rows.
// *narrow (set to 1 beforehand) is cleared when a count-1 row's integer value
// needs more than 32 bits.
__global__ void __launch_bounds__(256) k_split_count(const uint64_t* __restrict__ rows, uint64_t n, Layout S,
                                                     uint32_t* __restrict__ counts, uint64_t nblk,
                                                     uint64_t* __restrict__ narrow) {
    __shared__ uint32_t s_tmp[256 / 64 + 1];
    const uint64_t r0 = (uint64_t)blockIdx.x * SPLIT_T;
    uint32_t c = 0, cp = 0;
    bool wide = false;
    // the words a row is classified by, four rows' worth in flight per thread
    constexpr int G = 4;
    const bool pk = has_packed(S);
    for (uint32_t i0 = threadIdx.x; i0 < SPLIT_T; i0 += 256 * G) {
        uint64_t cv[G], sv[G], lo[G], hi[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint64_t r = r0 + i0 + (uint32_t)g * 256;
            cv[g] = 0;
            sv[g] = lo[g] = hi[g] = 0;
            if (r < n) {
                const uint64_t* q = rows + r * S.words;
                cv[g] = q[S.cnt];
                if (S.sum >= 0) {
                    sv[g] = q[S.sum];
                    lo[g] = q[S.mn];
                    hi[g] = q[S.mx];
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint64_t r = r0 + i0 + (uint32_t)g * 256;
            if (r >= n) continue;
            if (cv[g] == 1) {
                ++c;
                if (S.sum >= 0) wide |= !fits_i32(sv[g]);
            } else if (pk && (cv[g] >> 32) == 0 &&
                       (S.sum < 0 || (fits_i32(sv[g]) && fits_i32(lo[g]) && fits_i32(hi[g])))) {
                ++cp;
            }
        }
    }
    uint32_t tot, totp;
    block_exclusive_scan<256>(c, s_tmp, tot);
    block_exclusive_scan<256>(cp, s_tmp, totp);
    if (__syncthreads_or(wide) && threadIdx.x == 0) *narrow = 0;
    if (threadIdx.x == 0) {
        counts[blockIdx.x] = tot;
        counts[nblk + blockIdx.x] = totp;
    }
}

// offs[0..nblocks]: exclusive scan of the count-1 counts (offs[nblocks] = all
// count-1 rows), offs[nblocks + 1]: the narrow flag, offs[nblocks + 2]: all
// packed rows (written here), offs[nblocks + 3 ..]: the scan of the packed
// counts.  The run starts at out[0], or ends at out[end_words] when
// end_words is nonzero.
// A workgroup takes its SPLIT_T rows in tiles of SPLIT_TILE rows: a tile is
// loaded into LDS with consecutive threads on consecutive words, each thread
// then ranks the rows of its stripes (rows t, t + 256, ...) by ballots, the
// count-1 rows' columns and the packed rows leave in contiguous stores, and
// the other rows are copied word by word from LDS into their contiguous span
// of the run.
constexpr int SPLIT_TILE = 1024;
constexpr int SPLIT_MAXW = 6;
__global__ void __launch_bounds__(256) k_split_write(const uint64_t* __restrict__ rows, uint64_t n, Layout S,
                                                     Layout R, uint64_t* __restrict__ offs, uint64_t nblocks,
                                                     uint64_t* __restrict__ out, uint64_t end_words,
                                                     uint64_t cap_words) {
    __shared__ uint64_t s_rows[SPLIT_TILE * SPLIT_MAXW];
    __shared__ uint16_t s_msrc[SPLIT_TILE];
    __shared__ uint32_t s_wave[8];
    constexpr int STRIPES = SPLIT_TILE / 256;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t W = (uint32_t)S.words, PW = (uint32_t)packed_words(S);
    const uint64_t* offs_p = offs + nblocks + 3;
    const uint64_t n_single = offs[nblocks], n_packed = offs_p[nblocks];
    const bool narrow = offs[nblocks + 1] != 0;
    if (blockIdx.x == 0 && tid == 0) offs[nblocks + 2] = n_packed;
    const uint64_t s_words = single_bytes(n_single, R, narrow) / 8;
    const uint64_t n_words = s_words + n_packed * PW + (n - n_single - n_packed) * W;
    // a run larger than the room it is written into is not written at all
    // (the caller sees its size and copies the rows some other way)
    if (cap_words && n_words > cap_words) return;
    if (end_words) out += end_words - n_words;
    uint64_t* key_c = out;
    uint64_t* fs_c = out + n_single;
    void* int_c = out + n_single * (R.fs >= 0 ? 2 : 1);
    uint64_t* packed = out + s_words;
    uint64_t* multi = packed + n_packed * PW;
    const uint64_t blk0 = (uint64_t)blockIdx.x * SPLIT_T;
    uint64_t so = offs[blockIdx.x];     // count-1 rows before the current tile
    uint64_t sop = offs_p[blockIdx.x];  // packed rows before the current tile
    for (uint64_t t0 = blk0; t0 < blk0 + SPLIT_T && t0 < n; t0 += SPLIT_TILE) {
        const uint32_t tn = (uint32_t)(n - t0 < (uint64_t)SPLIT_TILE ? n - t0 : (uint64_t)SPLIT_TILE);
        stage_words<256, 12>(s_rows, rows + t0 * W, tn * W, nullptr, 0);
        __syncthreads();
        // ranks of the count-1 and of the packed rows, stripe by stripe (row
        // order is stripe-major)
        uint32_t srank[STRIPES], prank[STRIPES];
        uint8_t kind[STRIPES];  // 1: count-1, 2: packed, 0: state row (or none)
        uint32_t before = 0, before_p = 0;  // rows of each kind in earlier stripes
#pragma unroll
        for (int i = 0; i < STRIPES; ++i) {
            const uint32_t r = (uint32_t)(i * 256 + tid);
            uint8_t kd = 0;
            if (r < tn) {
                const uint64_t* q = s_rows + r * W;
                kd = q[S.cnt] == 1 ? 1 : packable(q, S) ? 2 : 0;
            }
            kind[i] = kd;
            const uint64_t bal = __ballot(kd == 1), balp = __ballot(kd == 2);
            if (lane == 0) {
                s_wave[wv] = (uint32_t)__popcll(bal);
                s_wave[4 + wv] = (uint32_t)__popcll(balp);
            }
            __syncthreads();
            uint32_t wbase = 0, stot = 0, wbase_p = 0, stot_p = 0;
            for (int q = 0; q < 4; ++q) {
                wbase += q < wv ? s_wave[q] : 0u;
                stot += s_wave[q];
                wbase_p += q < wv ? s_wave[4 + q] : 0u;
                stot_p += s_wave[4 + q];
            }
            const uint64_t lt = (1ull << lane) - 1ull;
            srank[i] = before + wbase + (uint32_t)__popcll(bal & lt);
            prank[i] = before_p + wbase_p + (uint32_t)__popcll(balp & lt);
            before += stot;
            before_p += stot_p;
            __syncthreads();
        }
        const uint32_t t_single = before, t_packed = before_p;
        // consecutive ranks of a stripe are consecutive rows of their part, so
        // a wave's stores are contiguous
#pragma unroll
        for (int i = 0; i < STRIPES; ++i) {
            const uint32_t r = (uint32_t)(i * 256 + tid);
            const uint64_t* q = s_rows + r * W;
            if (kind[i] == 1) {
                const uint64_t o = so + srank[i];
                key_c[o] = q[0];
                if (R.fs >= 0) fs_c[o] = q[S.fs];
                if (R.sum >= 0) {
                    if (narrow) ((int32_t*)int_c)[o] = (int32_t)(int64_t)q[S.sum];
                    else ((uint64_t*)int_c)[o] = q[S.sum];
                }
            } else if (kind[i] == 2) {
                uint64_t* pr = packed + (sop + prank[i]) * PW;
                uint64_t fld[4];
                int nf = 0;
                if (S.cnt >= 0) fld[nf++] = q[S.cnt] & 0xffffffffull;
                if (S.sum >= 0) {
                    fld[nf++] = q[S.sum] & 0xffffffffull;
                    fld[nf++] = q[S.mn] & 0xffffffffull;
                    fld[nf++] = q[S.mx] & 0xffffffffull;
                }
                int wd = 0;
                pr[wd++] = q[0];
                if (S.fs >= 0) pr[wd++] = q[S.fs];
                for (int f = 0; f < nf; f += 2) pr[wd++] = fld[f] | (f + 1 < nf ? fld[f + 1] << 32 : 0ull);
            } else if (r < tn) {
                s_msrc[r - srank[i] - prank[i]] = (uint16_t)r;  // its rank among the state rows
            }
        }
        __syncthreads();
        // the state rows, word by word from LDS into their contiguous span
        const uint32_t t_multi = tn - t_single - t_packed;
        uint64_t* md = multi + (t0 - so - sop) * W;  // rows before the tile that stay state rows
        for (uint32_t x = tid; x < t_multi * W; x += 256) {
            const uint32_t j = x / W, wd = x - j * W;
            md[x] = s_rows[(uint32_t)s_msrc[j] * W + wd];
        }
        so += t_single;
        sop += t_packed;
        __syncthreads();  // the tile's LDS is reused by the next tile
    }
}

// Gather of a wide-merge window into one staging buffer of state rows.  A
// small persistent grid walks the window's tasks (run slices of at most
// GATHER_ROWS rows), reading pinned host memory through its device mapping
// (or device memory) with contiguous word loads, GATHER_LOADS in flight per
// thread.
// The reads in flight are kept few on purpose: a host read holds a
// memory-request slot for the whole link latency, and the window being
// reduced meanwhile slows down with every such read (its kernels run about
// three times slower beside a gather of 48 workgroups with eight loads in
// flight per thread than alone).  64 workgroups, eight per XCD, with four
// loads in flight per thread read the link fastest while the window keeps
// up (measured on the 100M-row spilling merge: 0.5 ms faster than 48
// workgroups; 72 to 96 workgroups, or eight loads in flight, slow the
// window's reduction more than they speed the reads).  Each workgroup
// alternates between loading a slice and expanding it, so a plain stream of
// the same reads would run about 10% faster.  Raw slices (count-1 rows) are
// staged in LDS and expanded to state rows on the way out.
constexpr int GATHER_NT = 256;
constexpr uint32_t GATHER_GRID = 64;
constexpr int GATHER_LOADS = 4;
__global__ void __launch_bounds__(GATHER_NT) k_gather(const GatherTask* __restrict__ tasks, uint32_t n_tasks,
                                                      Layout R, Layout S, uint64_t* __restrict__ dst) {
    __shared__ uint64_t s_raw[GATHER_ROWS * 4];
    const uint32_t sw = (uint32_t)S.words, rw = (uint32_t)R.words;
    for (uint32_t ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
        const GatherTask t = tasks[ti];
        uint64_t* __restrict__ out = dst + t.dst_row * sw;
        const uint64_t* __restrict__ in = t.src;
        if (t.raw == 3) {
            // packed rows: loaded into LDS with GATHER_LOADS loads in flight per
            // thread, then widened to state rows
            const uint32_t pw = (uint32_t)packed_words(S);
            const uint32_t words = t.n * pw;
            for (uint32_t i = threadIdx.x; i < words; i += GATHER_LOADS * GATHER_NT) {
                uint64_t r[GATHER_LOADS];
#pragma unroll
                for (int q = 0; q < GATHER_LOADS; ++q) {
                    const uint32_t x = i + q * GATHER_NT;
                    if (x < words) r[q] = in[x];
                }
#pragma unroll
                for (int q = 0; q < GATHER_LOADS; ++q) {
                    const uint32_t x = i + q * GATHER_NT;
                    if (x < words) s_raw[x] = r[q];
                }
            }
            __syncthreads();
            const uint32_t base = S.fs >= 0 ? 2u : 1u;
            const uint32_t owords = t.n * sw;
            for (uint32_t o = threadIdx.x; o < owords; o += GATHER_NT) {
                const uint32_t r = o / sw, c = o - r * sw;
                const uint64_t* x = s_raw + r * pw;
                // field number of a 32-bit column: count, sum, min, max
                int f = -1;
                if ((int)c == S.cnt) f = 0;
                else if ((int)c == S.sum) f = S.cnt >= 0 ? 1 : 0;
                else if ((int)c == S.mn) f = S.cnt >= 0 ? 2 : 1;
                else if ((int)c == S.mx) f = S.cnt >= 0 ? 3 : 2;
                uint64_t v;
                if (c == 0) {
                    v = x[0];
                } else if ((int)c == S.fs) {
                    v = x[1];
                } else {
                    const uint32_t h = (uint32_t)(x[base + (uint32_t)f / 2] >> (32 * (f & 1)));
                    v = (int)c == S.cnt ? (uint64_t)h : (uint64_t)(int64_t)(int32_t)h;
                }
                out[o] = v;
            }
            __syncthreads();  // s_raw is refilled by the next task
            continue;
        }
        if (!t.raw) {
            const uint32_t words = t.n * sw;
            uint32_t i = threadIdx.x;
            for (; i + (GATHER_LOADS - 1) * GATHER_NT < words; i += GATHER_LOADS * GATHER_NT) {
                uint64_t r[GATHER_LOADS];
#pragma unroll
                for (int q = 0; q < GATHER_LOADS; ++q) r[q] = in[i + q * GATHER_NT];
#pragma unroll
                for (int q = 0; q < GATHER_LOADS; ++q) out[i + q * GATHER_NT] = r[q];
            }
            for (; i < words; i += GATHER_NT) out[i] = in[i];
            continue;
        }
        // count-1 rows: the key column, the f64 column and the integer
        // column of the slice, loaded into raw rows in LDS with 8-byte loads,
        // GATHER_LOADS in flight per thread.  A 4-byte integer column is read in
        // 8-byte words; a slice that starts at an odd row starts in the upper
        // half of its first word (column starts are 8-byte aligned).
        const uint32_t n = t.n;
        const bool nar = t.raw == 2;
        const uint32_t odd = nar ? (uint32_t)(((uintptr_t)t.iv >> 2) & 1u) : 0u;
        const uint64_t* iw = (const uint64_t*)((const char*)t.iv - 4 * odd);
        const uint32_t e0 = n, e1 = e0 + (R.fs >= 0 ? n : 0u);
        const uint32_t e2 = e1 + (R.sum < 0 ? 0u : nar ? (n + odd + 1) / 2 : n);
        for (uint32_t i = threadIdx.x; i < e2; i += GATHER_LOADS * GATHER_NT) {
            uint64_t r[GATHER_LOADS];
#pragma unroll
            for (int q = 0; q < GATHER_LOADS; ++q) {
                const uint32_t x = i + q * GATHER_NT;
                if (x < e2) r[q] = x < e0 ? in[x] : x < e1 ? t.fv[x - e0] : iw[x - e1];
            }
#pragma unroll
            for (int q = 0; q < GATHER_LOADS; ++q) {
                const uint32_t x = i + q * GATHER_NT;
                if (x >= e2) continue;
                if (x < e0) {
                    s_raw[x * rw] = r[q];
                } else if (x < e1) {
                    s_raw[(x - e0) * rw + (uint32_t)R.fs] = r[q];
                } else if (!nar) {
                    s_raw[(x - e1) * rw + (uint32_t)R.sum] = r[q];
                } else {
                    // little endian: the lower half is the earlier row
                    const int lo = 2 * (int)(x - e1) - (int)odd;
                    if (lo >= 0) s_raw[(uint32_t)lo * rw + (uint32_t)R.sum] = (uint64_t)(int64_t)(int32_t)(uint32_t)r[q];
                    if (lo + 1 < (int)n)
                        s_raw[(uint32_t)(lo + 1) * rw + (uint32_t)R.sum] = (uint64_t)(int64_t)(int32_t)(uint32_t)(r[q] >> 32);
                }
            }
        }
        __syncthreads();
        const uint32_t owords = t.n * sw;
        for (uint32_t o = threadIdx.x; o < owords; o += GATHER_NT) {
            const uint32_t r = o / sw, c = o - r * sw;
            const uint64_t* x = s_raw + r * rw;
            uint64_t v;
            if (c == 0) v = x[0];
            else if ((int)c == S.cnt) v = 1;
            else if ((int)c == S.fs) v = x[R.fs];
            else v = x[R.sum];  // sum, min and max of one row are its value
            out[o] = v;
        }
        __syncthreads();  // s_raw is refilled by the next task
    }
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
                    const uint64_t* offs, uint64_t* dst, Layout L, hipStream_t st, const uint32_t* hist_self,
                    uint64_t* offs_out, uint64_t max_chunk_rows) {
    // Rows of up to 3 words: a chunk of at most 2048 rows is one tile of 2048
    // rows staged in LDS (48 KB, two workgroups per CU); longer chunks go in
    // tiles of 1536 rows (36 KB and 129 VGPRs, three workgroups per CU, so
    // that one workgroup's loads overlap another's ranking and stores: the
    // 100M-row partition passes run about 7% faster).  Up to 6 words (state
    // rows): tiles of 1024 rows.
    if (L.words <= 3 && max_chunk_rows && max_chunk_rows <= (uint64_t)(PART_NT * PART_IPT / 2))
        hipLaunchKernelGGL((k_scatter<3, PART_IPT / 2>), dim3(n_chunks), dim3(PART_NT), 0, st, regions, chunks,
                           splitters, offs, dst, L, hist_self, offs_out);
    else if (L.words <= 3)
        hipLaunchKernelGGL((k_scatter<3, 6>), dim3(n_chunks), dim3(PART_NT), 0, st, regions, chunks, splitters,
                           offs, dst, L, hist_self, offs_out);
    else if (L.words <= 6)
        hipLaunchKernelGGL((k_scatter<6, PART_IPT / 4>), dim3(n_chunks), dim3(PART_NT), 0, st, regions, chunks,
                           splitters, offs, dst, L, hist_self, offs_out);
    else
        hipLaunchKernelGGL((k_scatter<0, PART_IPT>), dim3(n_chunks), dim3(PART_NT), 0, st, regions, chunks,
                           splitters, offs, dst, L, hist_self, offs_out);
}
void launch_bucket_starts(const Region* regions, uint32_t n_regions, const uint64_t* offs, const uint64_t* bs_base,
                          uint64_t* bstart, hipStream_t st) {
    hipLaunchKernelGGL(k_bucket_starts, dim3(n_regions), dim3(256), 0, st, regions, offs, bs_base, bstart);
}
void launch_hist_batch(const Region& r, Region* reg, uint64_t* ctl, uint32_t ctl_words, const Chunk* chunks,
                       uint32_t n_chunks, const uint64_t* splitters, uint32_t* hist, hipStream_t st) {
    hipLaunchKernelGGL(k_hist_batch, dim3(n_chunks), dim3(PART_NT), 0, st, r, reg, ctl, ctl_words, chunks, splitters,
                       hist);
}
void launch_copy_words(const uint64_t* src, uint64_t* dst, uint64_t n, hipStream_t st) {
    if (!n) return;
    uint64_t g = (n + 1023) / 1024;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_copy_words, dim3((uint32_t)g), dim3(256), 0, st, src, dst, n);
}
void launch_extract_keys(const uint64_t* rows, uint64_t n, uint32_t stride, uint64_t* keys, hipStream_t st) {
    if (!n) return;
    uint64_t g = (n + 1023) / 1024;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_extract_keys, dim3((uint32_t)g), dim3(256), 0, st, rows, n, stride, keys);
}
void launch_sample_keys(ColView src, uint64_t n, uint64_t S, uint64_t* out, hipStream_t st) {
    if (!S) return;
    hipLaunchKernelGGL(k_sample_keys, dim3((uint32_t)((S + 255) / 256)), dim3(256), 0, st, src, n, S, out);
}
uint64_t sorted_tiles(uint64_t n) { return (n + SORTED_T - 1) / SORTED_T; }
void launch_sorted_tiles(ColView V, uint64_t n, int shift, uint32_t* heads, uint32_t* bad, hipStream_t st) {
    const uint64_t m = sorted_tiles(n);
    if (!m) return;
    hipLaunchKernelGGL(k_sorted_tiles, dim3((uint32_t)m), dim3(SORTED_NT), 0, st, V, n, shift, heads, bad);
}
void launch_sorted_align(ColView V, uint64_t n, int shift, uint64_t* bounds, hipStream_t st) {
    const uint64_t m = sorted_tiles(n);
    hipLaunchKernelGGL(k_sorted_align, dim3((uint32_t)((m + 1 + 255) / 256)), dim3(256), 0, st, V, n, shift, m, bounds);
}
void launch_sorted_ranges(ColView V, uint64_t n, int shift, const uint64_t* bounds, const uint64_t* offs, OutView out,
                          uint64_t cap, uint64_t* bigs, uint32_t* n_bigs, hipStream_t st) {
    const uint64_t m = sorted_tiles(n);
    if (!m) return;
    hipLaunchKernelGGL(k_sorted_ranges, dim3((uint32_t)m), dim3(SORTED_NT), 0, st, V, n, shift, bounds, offs, out, cap,
                       bigs, n_bigs);
}
void launch_sorted_big_final(ColView V, int shift, const uint64_t* bigs, uint32_t n_bigs, const uint32_t* first,
                             const void* partials, OutView out, uint64_t cap, hipStream_t st) {
    if (!n_bigs) return;
    hipLaunchKernelGGL(k_sorted_big_final, dim3(n_bigs), dim3(256), 0, st, V, shift, bigs, first, (const Agg*)partials,
                       out, cap);
}
void launch_fill(uint64_t* p, uint64_t n, uint64_t value, hipStream_t st) {
    if (!n) return;
    uint64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)g), dim3(256), 0, st, p, n, value);
}
void launch_leaf(const Leaf* leaves, uint32_t n_leaves, const uint32_t* leaf_dest, const uint32_t* first_seg,
                 const Dest* dests, const void* partials, uint64_t* status, uint64_t* totals, uint32_t* ctl,
                 hipStream_t st) {
    if (!n_leaves) return;
    hipLaunchKernelGGL(k_leaf, dim3(n_leaves), dim3(LEAF_NT), 0, st, leaves, leaf_dest, first_seg, dests,
                       (const Agg*)partials, status, totals, ctl);
}
void launch_leaf_flat(const FlatSlot* slots, uint32_t n_slots, const FlatInst* insts, const Region* regions,
                      const uint64_t* splitters, const uint64_t* offs, const uint64_t* part, Layout L,
                      const uint32_t* first_slot, const Dest* dests, uint64_t* status, uint64_t* totals,
                      uint32_t* ctl, hipStream_t st, const uint32_t* single_of, const void* partials,
                      uint32_t max_pieces, uint64_t* host_out) {
    if (!n_slots) return;
    hipLaunchKernelGGL(k_leaf_flat, dim3(n_slots), dim3(LEAF_NT), 0, st, slots, insts, regions, splitters, offs, part,
                       L, first_slot, dests, status, totals, ctl, single_of, (const Agg*)partials, max_pieces,
                       host_out);
}
void launch_flat_single_partial(const Region* regions, const uint64_t* offs, const uint64_t* part, Layout L,
                                const uint32_t* single_buckets, uint32_t n_single, uint32_t max_pieces, void* partials,
                                hipStream_t st) {
    if (!n_single) return;
    hipLaunchKernelGGL(k_flat_single_partial, dim3(n_single * max_pieces), dim3(256), 0, st, regions, offs, part, L,
                       single_buckets, max_pieces, (Agg*)partials);
}
void launch_single_partial(const Leaf* leaves, const SinglePiece* pieces, uint32_t n_pieces, void* partials,
                           hipStream_t st) {
    if (!n_pieces) return;
    hipLaunchKernelGGL(k_single_partial, dim3(n_pieces), dim3(256), 0, st, leaves, pieces, (Agg*)partials);
}
size_t single_partial_bytes() { return sizeof(Agg); }
uint64_t merge_parts(uint64_t na, uint64_t nb) { return (na + nb + MG_D - 1) / MG_D; }
// A, B, out: row-major state rows of layout L.  splits: 2*(parts+1) words;
// status: parts words and ctl: 2 words, both zeroed.
void launch_merge(const uint64_t* A, uint64_t na, const uint64_t* B, uint64_t nb, uint64_t* out, Layout L,
                  uint64_t* splits, uint64_t* status, uint32_t* ctl, uint64_t* total_out, hipStream_t st,
                  uint64_t* next_ctl, uint32_t next_words, uint64_t* host_out, uint64_t rev_cap) {
    const uint64_t parts = merge_parts(na, nb);
    if (parts == 0) return;
    hipLaunchKernelGGL(k_merge_splits, dim3((uint32_t)((parts + 1 + 255) / 256)), dim3(256), 0, st, A, na, B, nb,
                       (uint32_t)L.words, parts, splits);
    // a grid of at most MG_GRID workgroups leaves compute units to the batch
    // sort running beside the merge
    const uint32_t grid = (uint32_t)(parts < MG_GRID ? parts : MG_GRID);
    hipLaunchKernelGGL(k_merge, dim3(grid), dim3(MG_NT), 0, st, A, na, B, nb, splits, out, L, status, ctl, total_out,
                       next_ctl, next_words, (uint32_t)parts, host_out, rev_cap);
}
void launch_rs_probe(const uint64_t* U, const uint64_t* m_ptr, uint32_t w, const uint64_t* cur, uint64_t* p_out,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_rs_probe, dim3(1), dim3(64), 0, st, U, m_ptr, w, cur, p_out);
}
void launch_rs_evict(const uint64_t* U, uint64_t m, uint32_t w, uint64_t p, uint64_t a, uint64_t b, uint64_t* out,
                     uint64_t* cur, hipStream_t st) {
    if (!m) return;
    uint64_t g = (m + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_rs_evict, dim3((uint32_t)g), dim3(256), 0, st, U, m, w, p, a, b, out, cur);
}
void launch_scan(const uint32_t* in, uint64_t n, uint64_t* tile_sums, uint64_t* offs, hipStream_t st);
uint64_t split_blocks(uint64_t n) { return (n + SPLIT_T - 1) / SPLIT_T; }
// counts: 2 * split_blocks(n) words; tiles as for launch_scan; offs:
// 2 * split_blocks(n) + 4 words (the count-1 scan, the narrow flag, the packed
// rows' total, the packed scan; see k_split_write).
void launch_split(const uint64_t* rows, uint64_t n, Layout S, Layout R, uint32_t* counts, uint64_t* tiles,
                  uint64_t* offs, uint64_t* out, uint64_t end_words, hipStream_t st, uint64_t cap_words) {
    const uint64_t nb = split_blocks(n);
    if (!nb) return;
    // offs[nb + 1] (beyond the scan's entries) holds the narrow flag
    launch_fill(offs + nb + 1, 1, 1, st);
    hipLaunchKernelGGL(k_split_count, dim3((uint32_t)nb), dim3(256), 0, st, rows, n, S, counts, nb, offs + nb + 1);
    launch_scan(counts, nb, tiles, offs, st);
    launch_scan(counts + nb, nb, tiles, offs + nb + 3, st);
    hipLaunchKernelGGL(k_split_write, dim3((uint32_t)nb), dim3(256), 0, st, rows, n, S, R, offs, nb, out, end_words,
                       cap_words);
}
void launch_gather(const GatherTask* tasks, uint32_t n_tasks, Layout R, Layout S, uint64_t* dst, hipStream_t st) {
    if (!n_tasks) return;
    const uint32_t g = n_tasks < GATHER_GRID ? n_tasks : GATHER_GRID;
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(GATHER_NT), 0, st, tasks, n_tasks, R, S, dst);
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
        launch_fill(offs, 1, 0, st);
        return;
    }
    if (n <= SMALL_SCAN_MAX) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(SMALL_SCAN_NT), 0, st, in, n, offs);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)t), dim3(SCAN_NT), 0, st, in, n, tile_sums);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, tile_sums, t);
    hipLaunchKernelGGL(k_scan_final, dim3((uint32_t)t), dim3(SCAN_NT), 0, st, in, n, tile_sums, offs);
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
void launch_unpack_hi(const uint64_t* hi, uint64_t n, int32_t* a, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_unpack_hi, grid_rows(n), dim3(256), 0, st, hi, n, a);
}
void launch_unpack_pairs(const uint64_t* keys, uint64_t n, int32_t* a, int32_t* b, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_unpack_pairs, grid_rows(n), dim3(256), 0, st, keys, n, a, b);
}
void launch_unpack_pairs_at(const uint64_t* keys, uint64_t max_n, const uint64_t* lo, const uint64_t* hi,
                            uint64_t cap, int32_t* a, int32_t* b, hipStream_t st) {
    if (!max_n) return;
    hipLaunchKernelGGL(k_unpack_pairs_at, grid_rows(max_n), dim3(256), 0, st, keys, lo, hi, cap, a, b);
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

// ---------------------------------------------------------------------------
// Multi-column keys with offset-value codes (Section 2: the table of
// offset-value codes; Section 5: column accesses).  Rows are ordered on K
// signed int64 columns, lexicographically: a stable LSD radix sort of a row
// permutation, one column at a time from the last to the first, 8-bit digits
// of the column value relative to its minimum.  Each row of the sorted stream
// is then coded against its predecessor (offset = leading columns equal,
// value = the row's value in the first differing column); a row whose offset
// is below K starts a group, so the in-stream grouping takes one test per row
// and never compares more than K column values for a row.
// ---------------------------------------------------------------------------

constexpr int RDX_NT = 256;
constexpr int RDX_IPT = 16;
constexpr int RDX_TILE = RDX_NT * RDX_IPT;
constexpr uint64_t SIGN64 = 1ull << 63;

// min and max of a column as order-preserving unsigned values (x ^ 2^63);
// out[0] starts at ~0 and out[1] at 0
__global__ void __launch_bounds__(256) k_col_minmax(const int64_t* __restrict__ col, uint64_t n,
                                                    unsigned long long* __restrict__ out) {
    uint64_t lo = ~0ull, hi = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const uint64_t u = (uint64_t)col[i] ^ SIGN64;
        lo = u < lo ? u : lo;
        hi = u > hi ? u : hi;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&out[0], (unsigned long long)lo);
        atomicMax(&out[1], (unsigned long long)hi);
    }
}

// keys[i] = the column value of row perm[i] (row i without a permutation),
// as an unsigned offset from the column's minimum
__global__ void k_col_keys(const int64_t* __restrict__ col, const uint32_t* __restrict__ perm, uint64_t n,
                           uint64_t lo, uint64_t* __restrict__ keys) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = perm ? perm[i] : i;
        keys[i] = ((uint64_t)col[r] ^ SIGN64) - lo;
    }
}

// digit counts of each tile, digit-major: hist[d * nblocks + b]
__global__ void __launch_bounds__(RDX_NT) k_rdx_hist(const uint64_t* __restrict__ keys, uint64_t n, int shift,
                                                    uint32_t nblocks, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * RDX_TILE;
    for (int j = 0; j < RDX_IPT; ++j) {
        const uint64_t e = t0 + (uint64_t)j * RDX_NT + threadIdx.x;
        if (e < n) atomicAdd(&h[(uint32_t)(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one digit pass.  A tile is taken in 16 rounds of 256
// consecutive rows; a row's rank is the rows of its digit in earlier rounds,
// in earlier waves of its round and in earlier lanes of its wave.
__global__ void __launch_bounds__(RDX_NT) k_rdx_scatter(const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ perm, uint64_t n, int shift,
                                                       uint32_t nblocks, const uint64_t* __restrict__ offs,
                                                       uint64_t* __restrict__ keys_out,
                                                       uint32_t* __restrict__ perm_out) {
    __shared__ uint32_t cnt[256];
    __shared__ uint32_t wc[RDX_NT / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    cnt[tid] = 0;
    for (int q = 0; q < RDX_NT / 64; ++q) wc[q][tid] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * RDX_TILE;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int j = 0; j < RDX_IPT; ++j) {
        const uint64_t e = t0 + (uint64_t)j * RDX_NT + tid;
        const bool ok = e < n;
        const uint64_t key = ok ? keys[e] : 0;
        const uint32_t p = ok ? (perm ? perm[e] : (uint32_t)e) : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint64_t match = wave_match(d, 8, __ballot(ok));
        const uint32_t before = (uint32_t)__popcll(match & lt);
        if (ok && before == 0) wc[w][d] = (uint32_t)__popcll(match);
        __syncthreads();
        if (ok) {
            uint32_t r = cnt[d] + before;
            for (int q = 0; q < w; ++q) r += wc[q][d];
            const uint64_t pos = offs[(uint64_t)d * nblocks + blockIdx.x] + r;
            keys_out[pos] = key;
            perm_out[pos] = p;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int q = 0; q < RDX_NT / 64; ++q) {
            add += wc[q][tid];
            wc[q][tid] = 0;
        }
        cnt[tid] += add;
        __syncthreads();
    }
}

// Offset-value code of every row of the sorted stream against its
// predecessor (the first row: offset 0, against a base that differs in the
// first column); heads[i] = 1 when the offset is below K.  Column values
// compared are summed into *compares.
__global__ void __launch_bounds__(256) k_ovc(const int64_t* const* __restrict__ cols, uint32_t K,
                                             const uint32_t* __restrict__ perm, uint64_t n,
                                             uint32_t* __restrict__ heads, uint32_t* __restrict__ code_off,
                                             int64_t* __restrict__ code_val,
                                             unsigned long long* __restrict__ compares) {
    uint64_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const uint32_t a = perm ? perm[i] : (uint32_t)i;
        uint32_t off = 0;
        if (i > 0) {
            const uint32_t b = perm ? perm[i - 1] : (uint32_t)(i - 1);
            while (off < K && cols[off][a] == cols[off][b]) ++off;
            acc += off < K ? off + 1 : K;
        }
        heads[i] = off < K ? 1u : 0u;
        if (code_off) code_off[i] = off;
        if (code_val) code_val[i] = off < K ? cols[off][a] : 0;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(compares, (unsigned long long)acc);
}

// group number of every sorted row (heads scanned: offs exclusive), the
// sorted position of each group's first row, and the value column in
// sorted order
__global__ void k_group_ids(const uint32_t* __restrict__ heads, const uint64_t* __restrict__ offs,
                            const uint32_t* __restrict__ perm, const int64_t* __restrict__ v, uint64_t n,
                            uint64_t* __restrict__ gid, uint64_t* __restrict__ head_pos,
                            int64_t* __restrict__ v_sorted) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t g = offs[i] + heads[i] - 1;
        gid[i] = g;
        if (heads[i]) head_pos[g] = i;
        if (v) v_sorted[i] = v[perm ? perm[i] : i];
    }
}

// key columns of every group from its first row
__global__ void k_group_keys(const int64_t* const* __restrict__ cols, uint32_t K, const uint32_t* __restrict__ perm,
                             const uint64_t* __restrict__ head_pos, uint64_t groups,
                             int64_t* const* __restrict__ out_cols) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t r = perm ? perm[head_pos[g]] : (uint32_t)head_pos[g];
        for (uint32_t c = 0; c < K; ++c) out_cols[c][g] = cols[c][r];
    }
}

static dim3 grid_of(uint64_t n, uint64_t cap) {
    uint64_t g = (n + 255) / 256;
    if (g > cap) g = cap;
    return dim3((uint32_t)(g ? g : 1));
}

uint64_t rdx_blocks(uint64_t n) { return (n + RDX_TILE - 1) / RDX_TILE; }
void launch_col_minmax(const int64_t* col, uint64_t n, uint64_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_col_minmax, grid_of(n, 2048), dim3(256), 0, st, col, n, (unsigned long long*)out);
}
void launch_col_keys(const int64_t* col, const uint32_t* perm, uint64_t n, uint64_t lo, uint64_t* keys,
                     hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_col_keys, grid_of(n, 16384), dim3(256), 0, st, col, perm, n, lo, keys);
}
void launch_rdx_hist(const uint64_t* keys, uint64_t n, int shift, uint32_t* hist, hipStream_t st) {
    const uint64_t nb = rdx_blocks(n);
    if (!nb) return;
    hipLaunchKernelGGL(k_rdx_hist, dim3((uint32_t)nb), dim3(RDX_NT), 0, st, keys, n, shift, (uint32_t)nb, hist);
}
void launch_rdx_scatter(const uint64_t* keys, const uint32_t* perm, uint64_t n, int shift, const uint64_t* offs,
                        uint64_t* keys_out, uint32_t* perm_out, hipStream_t st) {
    const uint64_t nb = rdx_blocks(n);
    if (!nb) return;
    hipLaunchKernelGGL(k_rdx_scatter, dim3((uint32_t)nb), dim3(RDX_NT), 0, st, keys, perm, n, shift, (uint32_t)nb,
                       offs, keys_out, perm_out);
}
void launch_ovc(const int64_t* const* cols, uint32_t K, const uint32_t* perm, uint64_t n, uint32_t* heads,
                uint32_t* code_off, int64_t* code_val, uint64_t* compares, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_ovc, grid_of(n, 16384), dim3(256), 0, st, cols, K, perm, n, heads, code_off, code_val,
                       (unsigned long long*)compares);
}
void launch_group_ids(const uint32_t* heads, const uint64_t* offs, const uint32_t* perm, const int64_t* v,
                      uint64_t n, uint64_t* gid, uint64_t* head_pos, int64_t* v_sorted, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_group_ids, grid_of(n, 16384), dim3(256), 0, st, heads, offs, perm, v, n, gid, head_pos,
                       v_sorted);
}
void launch_group_keys(const int64_t* const* cols, uint32_t K, const uint32_t* perm, const uint64_t* head_pos,
                       uint64_t groups, int64_t* const* out_cols, hipStream_t st) {
    if (!groups) return;
    hipLaunchKernelGGL(k_group_keys, grid_of(groups, 16384), dim3(256), 0, st, cols, K, perm, head_pos, groups,
                       out_cols);
}

// ---------------------------------------------------------------------------
// Library-owned scratch for callers that cannot allocate: a file-scope device
// array that each GPU the library runs on holds until the process ends.  Its
// device address differs per GPU and is looked up once per device, with that
// device current; host code uses only the looked-up address, never the
// array's name (a host-side stand-in).
// ---------------------------------------------------------------------------

static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the device must be current
        void* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr || ((uintptr_t)ptr & 255)) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace isa
