// Host engine: workspace carving and the multi-level partition driver that
// sorts and reduces many independent instances at once.
//
// A "sort-reduce" call takes unsorted rows (raw input rows or state rows) of
// one or more instances and produces, per instance, its sorted unique state
// rows.  Each instance is split into key ranges by sampled splitters (one
// level of an ordered index per pass, Section 3.3), ranges too large for one
// workgroup are split again, and every final range is sorted and reduced in
// LDS (Section 6.1: the batch is sorted within the cache and duplicates
// collapse; Section 2.1: in-stream grouping of sorted rows).
#include "isa_engine.h"

#include <algorithm>
#include <functional>
#include <cstring>

#include "../../include/insort.h"

namespace isa {

static void ck(hipError_t e, const char* what) {
    if (e != hipSuccess) throw Fail{ISA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

Layout raw_layout(const Cols& k) {
    Layout L;
    L.words = 1;
    L.cnt = L.sum = L.mn = L.mx = L.fs = -1;
    if (k.v) L.sum = L.mn = L.mx = L.words++;
    if (k.f) L.fs = L.words++;
    return L;
}

Layout state_layout(const Cols& k) {
    Layout L;
    L.words = 1;
    L.cnt = L.sum = L.mn = L.mx = L.fs = -1;
    if (k.c) L.cnt = L.words++;
    if (k.v) {
        L.sum = L.words++;
        L.mn = L.words++;
        L.mx = L.words++;
    }
    if (k.f) L.fs = L.words++;
    return L;
}

ColView aos_view(const uint64_t* base, const Layout& L) {
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

OutView aos_out(uint64_t* base, const Layout& L) {
    OutView v;
    v.key = base;
    v.cnt = L.cnt >= 0 ? base + L.cnt : nullptr;
    v.sum = L.sum >= 0 ? (int64_t*)(base + L.sum) : nullptr;
    v.mn = L.mn >= 0 ? (int64_t*)(base + L.mn) : nullptr;
    v.mx = L.mx >= 0 ? (int64_t*)(base + L.mx) : nullptr;
    v.fs = L.fs >= 0 ? (double*)(base + L.fs) : nullptr;
    v.stride = (uint64_t)L.words;
    return v;
}

void* Arena::take(uint64_t bytes) {
    uint64_t o = (off + 255) & ~(uint64_t)255;
    if (o + bytes > cap)
        throw Fail{ISA_EBUDGET, "workspace exhausted: need " + std::to_string(o + bytes) + " of " +
                                    std::to_string(cap) + " bytes (" + std::to_string(bytes) + " at " +
                                    std::to_string(o) + ")"};
    off = o + bytes;
    if (off > peak) peak = off;
    return base + o;
}

// ---------------------------------------------------------------------------
// Engine: pinned staging with a bump pointer that resets at every sync.
// ---------------------------------------------------------------------------

void* Engine::pinned_buf(uint64_t bytes) {
    uint64_t need = ((pinned_used + 255) & ~(uint64_t)255) + bytes;
    if (need > pinned_cap) {
        if (no_alloc) throw Fail{ISA_ENOMEM, "pinned staging would grow"};
        // Older buffers may still be the target of copies in flight or hold
        // readbacks not yet consumed: retire them, free them at destruction.
        uint64_t cap = pinned_cap ? 2 * pinned_cap : (8u << 20);
        while (cap < bytes + 256) cap *= 2;
        if (pinned) retired.push_back(pinned);
        pinned = nullptr;
        ck(hipHostMalloc((void**)&pinned, cap, 0), "hipHostMalloc(staging)");
        pinned_cap = cap;
        pinned_used = 0;
    }
    uint64_t o = (pinned_used + 255) & ~(uint64_t)255;
    pinned_used = o + bytes;
    return pinned + o;
}

static hipEvent_t pool_event(Engine& E) {
    if (E.ev_used == E.ev_pool.size()) {
        if (E.no_alloc) throw Fail{ISA_ENOMEM, "profiling events would be created"};
        hipEvent_t e;
        ck(hipEventCreate(&e), "hipEventCreate");
        E.ev_pool.push_back(e);
    }
    return E.ev_pool[E.ev_used++];
}

void Engine::pbegin(const char* name, hipStream_t st) {
    if (!prof_on) return;
    ProfRec r;
    r.name = name;
    r.a = pool_event(*this);
    r.b = pool_event(*this);
    r.rows = r.bytes = 0;
    ck(hipEventRecord(r.a, st ? st : stream), "hipEventRecord");
    prof.push_back(r);
}

void Engine::pend(uint64_t rows, uint64_t bytes, hipStream_t st) {
    if (!prof_on) return;
    ProfRec& r = prof.back();
    r.rows = rows;
    r.bytes = bytes;
    ck(hipEventRecord(r.b, st ? st : stream), "hipEventRecord");
}

hipStream_t Engine::copier() {
    if (!copy_stream && no_alloc) throw Fail{ISA_ENOMEM, "a copy stream would be created"};
    if (!copy_stream) ck(hipStreamCreateWithFlags(&copy_stream, hipStreamNonBlocking), "hipStreamCreate");
    return copy_stream;
}

hipStream_t Engine::side(int i) {
    if (!side_streams[i] && no_alloc) throw Fail{ISA_ENOMEM, "a side stream would be created"};
    if (!side_streams[i]) ck(hipStreamCreateWithFlags(&side_streams[i], hipStreamNonBlocking), "hipStreamCreate");
    return side_streams[i];
}

hipStream_t Engine::capturer() {
    if (!capture_stream && no_alloc) throw Fail{ISA_ENOMEM, "a capture stream would be created"};
    if (!capture_stream) ck(hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking), "hipStreamCreate");
    return capture_stream;
}

hipEvent_t Engine::sync_event(size_t i) {
    while (sync_events.size() <= i) {
        if (no_alloc) throw Fail{ISA_ENOMEM, "an event would be created"};
        hipEvent_t e;
        ck(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
        sync_events.push_back(e);
    }
    return sync_events[i];
}

char* Engine::ring_slot(size_t i) {
    constexpr size_t SLOTS = 64;
    if (!ring && no_alloc) throw Fail{ISA_ENOMEM, "the readback ring would be allocated"};
    if (!ring) ck(hipHostMalloc((void**)&ring, SLOTS * 64, 0), "hipHostMalloc(ring)");
    return ring + (i % SLOTS) * 64;
}

uint64_t* Engine::ring_dev(size_t i) {
    char* h = ring_slot(i);
    if (!ring_dev_base) {
        void* d = nullptr;
        ck(hipHostGetDevicePointer(&d, ring, 0), "hipHostGetDevicePointer(ring)");
        ring_dev_base = (char*)d;
    }
    return (uint64_t*)(ring_dev_base + (h - ring));
}

// The caller guarantees that no copy from the previous table is in flight.
void* Engine::table_buf(uint64_t bytes) {
    if (bytes > table_cap) {
        if (no_alloc) throw Fail{ISA_ENOMEM, "the task table would grow"};
        if (table) hipHostFree(table);
        table = nullptr;
        table_cap = 0;
        uint64_t cap = 1u << 20;
        while (cap < bytes) cap *= 2;
        ck(hipHostMalloc((void**)&table, cap, 0), "hipHostMalloc(table)");
        table_cap = cap;
    }
    return table;
}

void Engine::prepare_no_alloc() {
    (void)ring_dev(0);
    if (pinned_cap < NOALLOC_PINNED_BYTES) {
        (void)pinned_buf(NOALLOC_PINNED_BYTES - 256);
        pinned_used = 0;
    }
    (void)sync_event(NOALLOC_EVENTS - 1);
}

void Engine::release() {
    if (ring) hipHostFree(ring);
    ring = nullptr;
    ring_dev_base = nullptr;
    if (table) hipHostFree(table);
    table = nullptr;
    table_cap = 0;
    if (copy_stream) hipStreamDestroy(copy_stream);
    copy_stream = nullptr;
    for (hipStream_t& st : side_streams) {
        if (st) hipStreamDestroy(st);
        st = nullptr;
    }
    if (capture_stream) hipStreamDestroy(capture_stream);
    capture_stream = nullptr;
    for (hipEvent_t e : sync_events) hipEventDestroy(e);
    sync_events.clear();
    for (hipEvent_t e : ev_pool) hipEventDestroy(e);
    ev_pool.clear();
    prof.clear();
    ev_used = 0;
    for (char* p : retired) hipHostFree(p);
    retired.clear();
    if (pinned) hipHostFree(pinned);
    pinned = nullptr;
    pinned_cap = pinned_used = 0;
}

void Engine::upload(void* dev, const void* host, uint64_t bytes) {
    if (!bytes) return;
    void* p = pinned_buf(bytes);
    std::memcpy(p, host, bytes);
    ck(hipMemcpyAsync(dev, p, bytes, hipMemcpyHostToDevice, stream), "hipMemcpyAsync(H2D)");
}

void Engine::sync() {
    ck(hipStreamSynchronize(stream), "hipStreamSynchronize");
    pinned_used = 0;
}

void Engine::drain() {
    for (hipStream_t st : {stream, copy_stream, side_streams[0], side_streams[1], side_streams[2], capture_stream})
        if (st) (void)hipStreamSynchronize(st);
}

// Device-to-host copy into pinned staging; the data is valid after sync() and
// until the next upload/download.
const void* download_async(Engine& E, const void* dev, uint64_t bytes) {
    if (!bytes) return nullptr;
    void* p = E.pinned_buf(bytes);
    ck(hipMemcpyAsync(p, dev, bytes, hipMemcpyDeviceToHost, E.stream), "hipMemcpyAsync(D2H)");
    return p;
}

// ---------------------------------------------------------------------------
// sort_reduce
// ---------------------------------------------------------------------------

uint64_t UpPack::add(const void* src, uint64_t bytes) {
    const uint64_t o = (total + 255) & ~(uint64_t)255;
    parts.push_back(Part{src, bytes, o});
    total = o + bytes;
    return o;
}

char* UpPack::commit(Engine& E, Arena& A) {
    char* dev = (char*)A.take(total ? total : 1);
    if (!total) return dev;
    char* host = (char*)E.pinned_buf(total);
    for (const Part& p : parts)
        if (p.bytes) std::memcpy(host + p.off, p.src, p.bytes);
    ck(hipMemcpyAsync(dev, host, total, hipMemcpyHostToDevice, E.stream), "hipMemcpyAsync(H2D)");
    return dev;
}

namespace {

struct Node {
    int kind;  // 0 sort leaf, 1 single-key leaf, 2 pending region, 3 expanded region
    ColView src;
    uint64_t n, pos, lo, hi;
    uint32_t inst;
    // an expanded region's buckets: pool[first_kid, first_kid + n_kids), in key order
    int first_kid = 0, n_kids = 0;
};

}  // namespace

uint32_t buckets_for(const Engine& E, uint64_t n) {
    const uint64_t t = E.tune.leaf_rows;
    uint64_t nb = (n + t - 1) / t;
    if (nb < 2) nb = 2;
    if (nb > MAX_BUCKETS) nb = MAX_BUCKETS;
    return (uint32_t)nb;
}

// Rows per partition chunk: at least min_rows (a multiple of PART_CHUNK_MIN)
// for small regions (more workgroups), up to four tiles for large ones.
uint64_t chunk_rows(const Engine& E, uint64_t n, uint64_t min_rows) {
    const uint64_t crow = (n / E.tune.chunk_split + min_rows - 1) / min_rows * min_rows;
    return std::max<uint64_t>(min_rows, std::min<uint64_t>(PART_CHUNK, crow));
}

// Least-significant-digit radix sort of host keys, 8 bits a pass; a pass
// whose digit is the same in every key is skipped.  (The splitter sample is
// sorted on the host before the first batch can start: about three times
// faster than a comparison sort for 32768 keys.)
static void sort_keys_host(std::vector<uint64_t>& a) {
    const size_t n = a.size();
    if (n < 2) return;
    std::vector<uint32_t> cnt(8 * 256, 0);
    for (uint64_t v : a)
        for (int d = 0; d < 8; ++d) ++cnt[d * 256 + ((v >> (8 * d)) & 255)];
    std::vector<uint64_t> b(n);
    for (int d = 0; d < 8; ++d) {
        uint32_t* c = &cnt[d * 256];
        if (c[(a[0] >> (8 * d)) & 255] == n) continue;
        uint32_t sum = 0;
        for (int i = 0; i < 256; ++i) {
            const uint32_t t = c[i];
            c[i] = sum;
            sum += t;
        }
        for (uint64_t v : a) b[c[(v >> (8 * d)) & 255]++] = v;
        a.swap(b);
    }
}

// Splitters for every batch of one input, from a stratified sample of
// WIDE_SAMPLE keys sorted on the host.  A heavy key (at least one bucket's
// share of the sample) gets a bucket of its own, [key, key+1); the light keys
// share the remaining buckets evenly by sample count.  A bucket boundary never
// falls inside a run of equal keys.
void choose_splitters(Engine& E, Arena& A, const ColView& src, uint64_t n, uint32_t nb, uint64_t* dev_out,
                      std::vector<uint64_t>& host_out, std::vector<double>* share, double* light_share) {
    constexpr uint64_t WIDE_SAMPLE = 32768;
    const uint64_t mark = A.off;
    const uint64_t S = std::min<uint64_t>(n, WIDE_SAMPLE);
    uint64_t* d_s = A.take_n<uint64_t>(S + 1);
    E.pbegin("k_sample");
    launch_sample_keys(src, n, S, d_s, E.stream);
    E.pend(S, S * 8);
    const uint64_t* h = (const uint64_t*)download_async(E, d_s, S * sizeof(uint64_t));
    E.sync();
    std::vector<uint64_t> x(h, h + S);
    sort_keys_host(x);
    // runs of equal keys in the sample
    std::vector<std::pair<uint64_t, uint64_t>> runs;  // (key, count)
    for (uint64_t i = 0; i < S;) {
        uint64_t j = i;
        while (j < S && x[j] == x[i]) ++j;
        runs.push_back({x[i], j - i});
        i = j;
    }
    // heavy: at least a bucket's share, and among the nb/4 largest runs (so
    // that light keys keep at least half of the buckets)
    uint64_t heavy_at = std::max<uint64_t>(1, S / nb);
    {
        std::vector<uint64_t> cnt;
        for (const auto& r : runs) cnt.push_back(r.second);
        const size_t top = nb / 4;
        if (cnt.size() > top && top > 0) {
            std::nth_element(cnt.begin(), cnt.begin() + (top - 1), cnt.end(), std::greater<uint64_t>());
            heavy_at = std::max(heavy_at, cnt[top - 1] + 1);
        }
    }
    uint64_t n_heavy = 0, light = 0;
    for (const auto& r : runs) {
        if (r.second >= heavy_at) ++n_heavy;
        else light += r.second;
    }
    // buckets: two boundaries per heavy key at most, the rest for light keys
    const uint64_t light_buckets = nb > 2 * n_heavy + 1 ? nb - 2 * n_heavy : 1;
    uint64_t target = std::max<uint64_t>(1, (light + light_buckets - 1) / light_buckets);
    std::vector<uint64_t> spl;
    // Greedy packing wastes part of some buckets; when it wants more
    // boundaries than there are, the surplus keys would all land in the last
    // bucket, so the light target grows until every boundary fits.
    for (;;) {
        spl.clear();
        uint64_t acc = 0, wanted = 0;
        auto cut = [&](uint64_t key) {  // a boundary below `key`
            if (spl.size() + 1 < nb && key > 0 && (spl.empty() || spl.back() < key)) spl.push_back(key);
        };
        for (const auto& r : runs) {
            if (r.second >= heavy_at) {
                cut(r.first);
                if (r.first != ~0ull) cut(r.first + 1);
                wanted += 2;
                acc = 0;
                continue;
            }
            if (acc > 0 && acc + r.second > target) {
                cut(r.first);
                ++wanted;
                acc = 0;
            }
            acc += r.second;
        }
        if (wanted + 1 <= nb || target >= S) break;
        target += std::max<uint64_t>(1, target / 16);
    }
    host_out.assign(MAX_BUCKETS - 1, ~0ull);
    for (size_t i = 0; i < spl.size() && i < (size_t)(nb - 1); ++i) host_out[i] = spl[i];
    std::vector<double> sh(nb, 0.0);
    for (const auto& r : runs) {
        const size_t b = std::upper_bound(spl.begin(), spl.end(), r.first) - spl.begin();
        sh[std::min<size_t>(b, nb - 1)] += (double)r.second / (double)S;
    }
    if (light_share) {
        // the largest sampled share of a bucket spanning more than one key
        double m = 0;
        for (uint32_t b = 0; b < nb; ++b) {
            const uint64_t lo = b ? host_out[b - 1] : 0ull;
            const uint64_t hi = b + 1 < nb ? host_out[b] - 1 : ~0ull;
            if (lo != hi) m = std::max(m, sh[b]);
        }
        *light_share = m;
    }
    if (share) *share = sh;
    E.upload(dev_out, host_out.data(), (MAX_BUCKETS - 1) * sizeof(uint64_t));
    E.sync();
    A.off = mark;
}

uint64_t sort_reduce_bytes(uint64_t rows, uint64_t n_inst, const Cols& k, bool state_rows) {
    const Layout L = state_rows ? state_layout(k) : raw_layout(k);
    const Layout S = state_layout(k);
    (void)S;
    return rows * (uint64_t)(2 * L.words) * 8 + rows * 4 + n_inst * 4608 + (4u << 20);
}

uint64_t flat_bytes(uint64_t rows, uint64_t n_inst, const Cols& k, bool state_rows) {
    const Layout L = state_rows ? state_layout(k) : raw_layout(k);
    // partition rows; per PART_TILE rows one histogram column of MAX_BUCKETS
    // counters and offsets and one chunk; per instance its splitters, slots,
    // status words and descriptors; 256-byte alignment of every block
    const uint64_t cols = rows / PART_TILE + n_inst;
    return rows * (uint64_t)L.words * 8 + cols * ((uint64_t)MAX_BUCKETS * 12 + sizeof(Chunk)) +
           n_inst * ((MAX_BUCKETS - 1) * 8 + (uint64_t)MAX_BUCKETS * (sizeof(FlatSlot) + 8) + sizeof(Region) +
                     sizeof(FlatInst) + sizeof(Dest) + 16) +
           (64u << 10);
}

std::vector<uint64_t> sort_reduce(Engine& E, Arena& A, const std::vector<Instance>& inst,
                                  const std::vector<Dest>& dests, const Cols& k, bool state_rows,
                                  const SplitterHint* hint) {
    const Layout L = state_rows ? state_layout(k) : raw_layout(k);
    // bytes of one source row as the caller's columns hold it
    const uint64_t src_row_bytes = (uint64_t)L.words * 8;
    std::vector<uint64_t> totals(dests.size(), 0);
    std::vector<Node> pool;
    uint64_t rows_all = 0;
    for (const Instance& x : inst) rows_all += x.n;
    // about one node per leaf of half a leaf's rows, plus the regions
    pool.reserve(inst.size() + 2 * (rows_all / (uint64_t)LEAF_CAP) * 2 + 1024);
    std::vector<int> roots(inst.size(), -1);
    uint64_t N = 0;
    bool need_part = false;
    for (size_t i = 0; i < inst.size(); ++i) {
        if (i > 0 && inst[i].dest < inst[i - 1].dest) throw Fail{ISA_EINVAL, "instances not ordered by dest"};
        if (inst[i].n == 0) continue;
        Node nd;
        nd.kind = inst[i].n <= (uint64_t)LEAF_CAP ? 0 : 2;
        nd.src = inst[i].src;
        nd.n = inst[i].n;
        nd.pos = N;
        nd.lo = 0;
        nd.hi = ~0ull;
        nd.inst = (uint32_t)i;
        roots[i] = (int)pool.size();
        pool.push_back(nd);
        N += inst[i].n;
        if (nd.kind == 2) need_part = true;
    }
    if (N == 0) return totals;

    uint64_t* P[2] = {nullptr, nullptr};
    if (need_part) P[0] = A.take_n<uint64_t>(N * (uint64_t)L.words);

    std::vector<int> pending;
    for (int r : roots)
        if (r >= 0 && pool[r].kind == 2) pending.push_back(r);

    int level = 0;
    while (!pending.empty()) {
        if (level >= 48) throw Fail{ISA_EDEVICE, "key-range partitioning did not converge"};
        if (!P[level & 1]) P[level & 1] = A.take_n<uint64_t>(N * (uint64_t)L.words);
        uint64_t* tgt = P[level & 1];
        std::vector<Region> regs;
        std::vector<Chunk> chunks;
        std::vector<uint64_t> bsb;
        uint64_t hist_total = 0, bs_total = 0;
        for (int id : pending) {
            const Node& nd = pool[id];
            Region r;
            r.src = nd.src;
            r.n = nd.n;
            r.out_pos = nd.pos;
            r.nb = buckets_for(E, nd.n);
            const uint64_t crow = chunk_rows(E, nd.n, PART_TILE);
            r.n_chunks = (uint32_t)((nd.n + crow - 1) / crow);
            r.hist_base = hist_total;
            hist_total += (uint64_t)r.nb * r.n_chunks;
            bsb.push_back(bs_total);
            bs_total += r.nb + 1;
            for (uint32_t c = 0; c < r.n_chunks; ++c) {
                Chunk ch;
                ch.region = (uint32_t)regs.size();
                ch.idx = c;
                ch.start = (uint64_t)c * crow;
                const uint64_t left = nd.n - ch.start;
                ch.n = (uint32_t)(left < crow ? left : crow);
                ch.pad = 0;
                chunks.push_back(ch);
            }
            regs.push_back(r);
        }
        const uint64_t mark = A.off;
        // one upload for the level's descriptors, one readback block for
        // splitters and bucket starts
        const bool fixed = hint && hint->dev && level == 0 && regs.size() == 1;
        if (fixed) regs[0].nb = hint->nb;
        if (fixed) {
            // recompute the histogram layout for the hinted bucket count
            hist_total = (uint64_t)regs[0].nb * regs[0].n_chunks;
            bs_total = regs[0].nb + 1;
        }
        UpPack up;
        const uint64_t o_regs = up.add(regs.data(), regs.size() * sizeof(Region));
        const uint64_t o_chunks = up.add(chunks.data(), chunks.size() * sizeof(Chunk));
        const uint64_t o_bsb = up.add(bsb.data(), bsb.size() * sizeof(uint64_t));
        char* d_up = up.commit(E, A);
        Region* d_regs = (Region*)(d_up + o_regs);
        Chunk* d_chunks = (Chunk*)(d_up + o_chunks);
        uint64_t* d_bsb = (uint64_t*)(d_up + o_bsb);
        const uint64_t spl_words = regs.size() * (MAX_BUCKETS - 1);
        uint64_t* d_rb = A.take_n<uint64_t>(spl_words + bs_total);
        uint64_t* d_spl = fixed ? (uint64_t*)hint->dev : d_rb;
        uint64_t* d_bstart = d_rb + spl_words;
        uint32_t* d_hist = A.take_n<uint32_t>(hist_total);
        uint64_t* d_offs = A.take_n<uint64_t>(hist_total + 1);
        uint64_t* d_tiles = A.take_n<uint64_t>(scan_tiles(hist_total) + 1);
        uint64_t lvl_rows = 0;
        for (const Region& r : regs) lvl_rows += r.n;
        const uint64_t in_bytes = (uint64_t)(level == 0 ? src_row_bytes : L.words * 8);
        if (!fixed) {
            E.pbegin("k_sample");
            launch_sample(d_regs, (uint32_t)regs.size(), d_spl, E.stream);
            E.pend(regs.size() * (uint64_t)SAMPLE_N, regs.size() * (uint64_t)SAMPLE_N * 8);
        }
        E.pbegin("k_hist");
        launch_hist(d_regs, d_chunks, (uint32_t)chunks.size(), d_spl, d_hist, E.stream);
        E.pend(lvl_rows, lvl_rows * 8);
        E.pbegin("k_scan");
        launch_scan(d_hist, hist_total, d_tiles, d_offs, E.stream);
        E.pend(hist_total, hist_total * 12);
        E.pbegin("k_scatter");
        launch_scatter(d_regs, d_chunks, (uint32_t)chunks.size(), d_spl, d_offs, tgt, L, E.stream);
        E.pend(lvl_rows, lvl_rows * in_bytes);
        launch_bucket_starts(d_regs, (uint32_t)regs.size(), d_offs, d_bsb, d_bstart, E.stream);
        ck(hipGetLastError(), "partition launch");
        const uint64_t* h_rb = (const uint64_t*)download_async(E, fixed ? d_bstart : d_rb,
                                                               ((fixed ? 0 : spl_words) + bs_total) * sizeof(uint64_t));
        E.sync();
        // read in place: the staging stays valid until the next sync
        const uint64_t* h_bs = fixed ? h_rb : h_rb + spl_words;
        const uint64_t* h_sp = fixed ? hint->host : h_rb;
        A.off = mark;
        std::vector<int> next;
        for (size_t ri = 0; ri < pending.size(); ++ri) {
            const int id = pending[ri];
            const Region& r = regs[ri];
            const uint64_t* sp = h_sp + ri * (MAX_BUCKETS - 1);
            const uint64_t* bs = h_bs + bsb[ri];
            if (bs[r.nb] != r.n) throw Fail{ISA_EDEVICE, "partition lost rows"};
            const int first_kid = (int)pool.size();
            for (uint32_t b = 0; b < r.nb; ++b) {
                const uint64_t size = bs[b + 1] - bs[b];
                if (!size) continue;
                uint64_t lo = b == 0 ? pool[id].lo : sp[b - 1];
                uint64_t hi = b + 1 == r.nb ? pool[id].hi : sp[b] - 1;
                if (lo < pool[id].lo) lo = pool[id].lo;
                if (hi > pool[id].hi) hi = pool[id].hi;
                Node c;
                c.pos = pool[id].pos + bs[b];
                c.src = aos_view(tgt + c.pos * (uint64_t)L.words, L);
                c.n = size;
                c.lo = lo;
                c.hi = hi;
                c.inst = pool[id].inst;
                c.kind = size <= (uint64_t)LEAF_CAP ? 0 : (lo == hi ? 1 : 2);
                if (c.kind == 2) next.push_back((int)pool.size());
                pool.push_back(c);
            }
            pool[id].first_kid = first_kid;
            pool[id].n_kids = (int)pool.size() - first_kid;
            pool[id].kind = 3;
        }
        pending.swap(next);
        ++level;
    }

    // Leaves in output order: instances in order, keys ascending within each.
    // They are written straight into pinned staging (at most one per node)
    // and uploaded from there.
    Leaf* const leaves = (Leaf*)E.pinned_buf(pool.size() * sizeof(Leaf));
    uint32_t* const leaf_dest = (uint32_t*)E.pinned_buf(pool.size() * sizeof(uint32_t));
    uint64_t nl = 0;
    std::vector<SinglePiece> pieces;
    std::vector<uint32_t> first_seg(dests.size() + 1, 0);
    std::vector<int> stack;
    uint32_t cur_dest = 0;
    for (size_t i = 0; i < inst.size(); ++i) {
        while (cur_dest < inst[i].dest) first_seg[++cur_dest] = (uint32_t)nl;
        if (roots[i] < 0) continue;
        stack.assign(1, roots[i]);
        while (!stack.empty()) {
            const int id = stack.back();
            stack.pop_back();
            const Node& nd = pool[id];
            if (nd.kind == 3) {
                for (int c = nd.first_kid + nd.n_kids - 1; c >= nd.first_kid; --c) stack.push_back(c);
                continue;
            }
            Leaf lf;
            lf.src = nd.src;
            lf.n = nd.n;
            lf.out_pos = nd.pos;
            lf.kind = (uint32_t)nd.kind;
            lf.single_first = 0;
            lf.single_count = 0;
            lf.pad = 0;
            if (nd.kind == 1) {
                lf.single_first = (uint32_t)pieces.size();
                for (uint64_t s = 0; s < nd.n; s += SINGLE_CHUNK) {
                    SinglePiece p;
                    p.leaf = (uint32_t)nl;
                    p.slot = (uint32_t)pieces.size();
                    p.start = s;
                    p.n = (uint32_t)std::min<uint64_t>(SINGLE_CHUNK, nd.n - s);
                    p.pad = 0;
                    pieces.push_back(p);
                }
                lf.single_count = (uint32_t)pieces.size() - lf.single_first;
            }
            leaves[nl] = lf;
            leaf_dest[nl] = inst[i].dest;
            ++nl;
        }
    }
    while (cur_dest < dests.size()) first_seg[++cur_dest] = (uint32_t)nl;

    Leaf* d_leaves = A.take_n<Leaf>(nl ? nl : 1);
    uint32_t* d_ldest = A.take_n<uint32_t>(nl ? nl : 1);
    if (nl) {
        ck(hipMemcpyAsync(d_leaves, leaves, nl * sizeof(Leaf), hipMemcpyHostToDevice, E.stream), "hipMemcpyAsync(leaves)");
        ck(hipMemcpyAsync(d_ldest, leaf_dest, nl * sizeof(uint32_t), hipMemcpyHostToDevice, E.stream),
           "hipMemcpyAsync(leaf destinations)");
    }
    UpPack up;
    const uint64_t o_first = up.add(first_seg.data(), first_seg.size() * sizeof(uint32_t));
    const uint64_t o_dests = up.add(dests.data(), dests.size() * sizeof(Dest));
    const uint64_t o_pieces = up.add(pieces.data(), pieces.size() * sizeof(SinglePiece));
    char* d_up = up.commit(E, A);
    uint32_t* d_first = (uint32_t*)(d_up + o_first);
    Dest* d_dests = (Dest*)(d_up + o_dests);
    SinglePiece* d_pieces = pieces.empty() ? nullptr : (SinglePiece*)(d_up + o_pieces);
    // control block: [ticket, error] word, per-dest totals, per-leaf status
    uint64_t* d_ctl = A.take_n<uint64_t>(1 + dests.size() + nl);
    uint64_t* d_totals = d_ctl + 1;
    uint64_t* d_status = d_totals + dests.size();
    void* d_partials = pieces.empty() ? nullptr : A.take(pieces.size() * single_partial_bytes());
    launch_fill(d_ctl, 1 + dests.size() + nl, 0, E.stream);
    uint64_t sort_rows = 0, single_rows = 0;
    for (uint64_t i = 0; i < nl; ++i) (leaves[i].kind == 0 ? sort_rows : single_rows) += leaves[i].n;
    const uint64_t leaf_bytes = need_part ? (uint64_t)L.words * 8 : src_row_bytes;
    if (!pieces.empty()) {
        E.pbegin("k_single");
        launch_single_partial(d_leaves, d_pieces, (uint32_t)pieces.size(), d_partials, E.stream);
        E.pend(single_rows, single_rows * leaf_bytes);
    }
    E.pbegin("k_leaf");
    launch_leaf(d_leaves, (uint32_t)nl, d_ldest, d_first, d_dests, d_partials, d_status, d_totals,
                (uint32_t*)d_ctl, E.stream);
    E.pend(sort_rows, sort_rows * leaf_bytes);
    ck(hipGetLastError(), "leaf launch");
    const uint64_t* h_ctl = (const uint64_t*)download_async(E, d_ctl, (1 + dests.size()) * sizeof(uint64_t));
    E.sync();
    if (h_ctl[0] >> 32) throw Fail{ISA_EDEVICE, "leaf placement wait timed out"};
    for (size_t d = 0; d < dests.size(); ++d) totals[d] = h_ctl[1 + d];
    return totals;
}

}  // namespace isa

namespace isa {

// Error word of a flat launch: bit 0 a timed-out wait (fatal), bit 1 an
// oversized bucket (the caller falls back to the general plan).
static bool finish_flat(const uint64_t* h_ctl, size_t n_dests, std::vector<uint64_t>& totals) {
    const uint64_t err = h_ctl[0] >> 32;
    if (err & 1) throw Fail{ISA_EDEVICE, "leaf placement wait timed out"};
    if (err & 2) return false;
    for (size_t d = 0; d < n_dests; ++d) totals[d] = h_ctl[1 + d];
    return true;
}

bool sort_reduce_flat(Engine& E, Arena& A, const std::vector<Instance>& inst, const std::vector<Dest>& dests,
                      const Cols& k, bool state_rows, const SplitterHint* hint, bool graph,
                      std::vector<uint64_t>& totals, uint64_t* ext_totals, const uint64_t** async_ctl) {
    if (async_ctl && graph) throw Fail{ISA_EINVAL, "internal: asynchronous flat plan with a graph"};
    const Layout L = state_rows ? state_layout(k) : raw_layout(k);
    totals.assign(dests.size(), 0);
    std::vector<Region> regs;
    std::vector<Chunk> chunks;
    std::vector<FlatInst> finst;
    std::vector<FlatSlot> slots;
    std::vector<uint32_t> first_slot(dests.size() + 1, 0);
    uint64_t N = 0, hist_total = 0;
    uint32_t cur_dest = 0;
    for (size_t i = 0; i < inst.size(); ++i) {
        const Instance& in = inst[i];
        if (i > 0 && in.dest < inst[i - 1].dest) throw Fail{ISA_EINVAL, "instances not ordered by dest"};
        if (in.n > FLAT_MAX) throw Fail{ISA_EINVAL, "instance too large for the flat plan"};
        while (cur_dest < in.dest) first_slot[++cur_dest] = (uint32_t)slots.size();
        if (in.n == 0) continue;
        if (in.n <= (uint64_t)LEAF_CAP) {
            FlatInst fi;
            fi.src = in.src;
            fi.n = in.n;
            slots.push_back(FlatSlot{0, (uint32_t)finst.size(), 0, in.dest});
            finst.push_back(fi);
            continue;
        }
        Region r;
        r.src = in.src;
        r.n = in.n;
        r.out_pos = N;
        r.nb = (hint && hint->dev && inst.size() == 1) ? hint->nb : buckets_for(E, in.n);
        const uint64_t crow = chunk_rows(E, in.n, PART_TILE);
        r.n_chunks = (uint32_t)((in.n + crow - 1) / crow);
        r.hist_base = hist_total;
        hist_total += (uint64_t)r.nb * r.n_chunks;
        for (uint32_t c = 0; c < r.n_chunks; ++c) {
            Chunk ch;
            ch.region = (uint32_t)regs.size();
            ch.idx = c;
            ch.start = (uint64_t)c * crow;
            const uint64_t left = in.n - ch.start;
            ch.n = (uint32_t)(left < crow ? left : crow);
            ch.pad = 0;
            chunks.push_back(ch);
        }
        for (uint32_t b = 0; b < r.nb; ++b) slots.push_back(FlatSlot{1, (uint32_t)regs.size(), b, in.dest});
        regs.push_back(r);
        N += in.n;
    }
    while (cur_dest < dests.size()) first_slot[++cur_dest] = (uint32_t)slots.size();
    if (slots.empty()) return true;
    const bool fixed = hint && hint->dev && regs.size() == 1;

    uint64_t* part = N ? A.take_n<uint64_t>(N * (uint64_t)L.words) : nullptr;
    uint64_t* d_spl = fixed ? (uint64_t*)hint->dev : A.take_n<uint64_t>(std::max<size_t>(1, regs.size()) * (MAX_BUCKETS - 1));
    uint32_t* d_hist = A.take_n<uint32_t>(hist_total + 1);
    uint64_t* d_offs = A.take_n<uint64_t>(hist_total + 1);
    uint64_t* d_ctl = A.take_n<uint64_t>(1 + dests.size() + slots.size());
    uint64_t* d_totals = ext_totals ? ext_totals : d_ctl + 1;
    uint64_t* d_status = d_ctl + 1 + dests.size();

    // descriptors are uploaded on the caller's stream before any capture
    UpPack up;
    const uint64_t o_regs = up.add(regs.data(), regs.size() * sizeof(Region));
    const uint64_t o_chunks = up.add(chunks.data(), chunks.size() * sizeof(Chunk));
    const uint64_t o_slots = up.add(slots.data(), slots.size() * sizeof(FlatSlot));
    const uint64_t o_inst = up.add(finst.data(), finst.size() * sizeof(FlatInst));
    const uint64_t o_first = up.add(first_slot.data(), first_slot.size() * sizeof(uint32_t));
    const uint64_t o_dests = up.add(dests.data(), dests.size() * sizeof(Dest));
    char* d_up = up.commit(E, A);
    Region* d_regs = (Region*)(d_up + o_regs);
    Chunk* d_chunks = (Chunk*)(d_up + o_chunks);
    uint64_t rows = 0;
    for (const Region& r : regs) rows += r.n;
    uint64_t leaf_rows = N;
    for (const FlatInst& fi : finst) leaf_rows += fi.n;
    // the kernels: launched directly on the caller's stream, or captured on a
    // private stream and launched as one graph on the caller's stream
    auto launches = [&](hipStream_t st) {
        launch_fill(d_ctl, 1 + dests.size() + slots.size(), 0, st);
        if (!regs.empty()) {
            if (!fixed) {
                E.pbegin("k_sample", st);
                launch_sample(d_regs, (uint32_t)regs.size(), d_spl, st);
                E.pend(regs.size() * (uint64_t)SAMPLE_N, regs.size() * (uint64_t)SAMPLE_N * 8, st);
            }
            E.pbegin("k_hist", st);
            launch_hist(d_regs, d_chunks, (uint32_t)chunks.size(), d_spl, d_hist, st);
            E.pend(rows, rows * 8, st);
            // no scan launch: a region of the flat plan has at most FLAT_MAX
            // rows, so every scatter workgroup sums its region's histogram
            // itself and writes its chunk's region-relative offsets
            E.pbegin("k_scatter", st);
            launch_scatter(d_regs, d_chunks, (uint32_t)chunks.size(), d_spl, d_offs, part, L, st, d_hist, d_offs);
            E.pend(rows, rows * (uint64_t)L.words * 8, st);
        }
        E.pbegin("k_leaf", st);
        launch_leaf_flat((FlatSlot*)(d_up + o_slots), (uint32_t)slots.size(), (FlatInst*)(d_up + o_inst), d_regs,
                         d_spl, d_offs, part, L, (uint32_t*)(d_up + o_first), (Dest*)(d_up + o_dests), d_status,
                         d_totals, (uint32_t*)d_ctl, st);
        E.pend(leaf_rows, leaf_rows * (uint64_t)L.words * 8, st);
    };
    if (graph) {
        hipStream_t cs = E.capturer();
        const bool prof = E.prof_on;
        E.prof_on = false;
        // the capture stream must see the upload: order it after the caller's stream
        ck(hipEventRecord(E.sync_event(8), E.stream), "hipEventRecord");
        ck(hipStreamWaitEvent(cs, E.sync_event(8), 0), "hipStreamWaitEvent");
        ck(hipStreamSynchronize(cs), "hipStreamSynchronize");
        hipGraph_t gr = nullptr;
        ck(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        launches(cs);
        const hipError_t ec = hipStreamEndCapture(cs, &gr);
        E.prof_on = prof;
        ck(ec, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            hipGraphDestroy(gr);
            ck(ei, "hipGraphInstantiate");
        }
        E.pbegin("graph_launch");
        const hipError_t el = hipGraphLaunch(ex, E.stream);
        E.pend(leaf_rows, 0);
        const uint64_t* h = (const uint64_t*)download_async(E, d_ctl, (1 + dests.size()) * sizeof(uint64_t));
        const hipError_t es = hipStreamSynchronize(E.stream);
        hipGraphExecDestroy(ex);
        hipGraphDestroy(gr);
        ck(el, "hipGraphLaunch");
        ck(es, "hipStreamSynchronize");
        E.sync();
        return finish_flat(h, dests.size(), totals);
    }
    launches(E.stream);
    ck(hipGetLastError(), "flat launch");
    const uint64_t* h_ctl = (const uint64_t*)download_async(E, d_ctl, (1 + dests.size()) * sizeof(uint64_t));
    if (async_ctl) {
        *async_ctl = h_ctl;
        totals.clear();
        return true;
    }
    E.sync();
    return finish_flat(h_ctl, dests.size(), totals);
}

// ---------------------------------------------------------------------------
// BatchProgram: run generation's per-batch sort-reduce with every descriptor
// uploaded once, so that a batch is a fixed sequence of launches.
// ---------------------------------------------------------------------------

namespace {
constexpr uint32_t BP_CTL_RING = 8;  // control blocks reused round-robin

}  // namespace

uint64_t batch_program_bytes(uint64_t Bt, const Cols& k) {
    const uint64_t ch = (Bt + PART_CHUNK_MIN - 1) / PART_CHUNK_MIN;  // the most chunks any tuning gives
    const uint64_t hist = (uint64_t)MAX_BUCKETS * ch;
    const uint64_t pieces = (Bt + SINGLE_CHUNK - 1) / SINGLE_CHUNK;
    const uint64_t desc = BP_CTL_RING * sizeof(Region) + 2 * ch * sizeof(Chunk) + MAX_BUCKETS * sizeof(FlatSlot) +
                          16 + 3 * sizeof(Dest) + BP_CTL_RING * (2 + MAX_BUCKETS) * 8 + 2 * MAX_BUCKETS * 4 +
                          BatchProgram::SETS * ((uint64_t)MAX_BUCKETS * pieces * single_partial_bytes() + 256) +
                          4 * 256;
    const uint64_t scratch = Bt * (uint64_t)raw_layout(k).words * 8 + hist * 4 + (hist + 1) * 8 + 8 * 256;
    // the scratch area also serves the general plan when a batch falls back
    return desc + 8 * 256 + std::max(BatchProgram::SETS * scratch, sort_reduce_bytes(Bt, 1, k, false));
}

void BatchProgram::setup(Engine& E, Arena& A, const ColView& src_rows, uint64_t n_rows, uint64_t batch_rows,
                         const Cols& k, const SplitterHint& hint, const std::vector<Dest>& dests) {
    n = n_rows;
    Bt = batch_rows;
    batches = (n + Bt - 1) / Bt;
    nb = hint.nb;
    L = raw_layout(k);
    src = src_rows;
    splitters = hint.dev;
    // a batch is one region: chunks of PART_CHUNK_MIN rows give every
    // compute unit a workgroup of the partition passes
    crow = chunk_rows(E, Bt, PART_CHUNK_MIN);
    chunks_full = (uint32_t)((Bt + crow - 1) / crow);
    const uint64_t last_n = n - (batches - 1) * Bt;
    chunks_last = (uint32_t)((last_n + crow - 1) / crow);
    auto chunk_list = [&](uint64_t bn, uint32_t cnt) {
        std::vector<Chunk> v(cnt);
        for (uint32_t c = 0; c < cnt; ++c) {
            v[c].region = 0;
            v[c].idx = c;
            v[c].start = (uint64_t)c * crow;
            const uint64_t left = bn - v[c].start;
            v[c].n = (uint32_t)(left < crow ? left : crow);
            v[c].pad = 0;
        }
        return v;
    };
    const std::vector<Chunk> cf = chunk_list(Bt < n ? Bt : n, chunks_full);
    const std::vector<Chunk> cl = chunk_list(last_n, chunks_last);
    std::vector<FlatSlot> slots(nb);
    for (uint32_t b = 0; b < nb; ++b) slots[b] = FlatSlot{1, 0, b, 0};
    const uint32_t first[2] = {0, nb};
    // single-key buckets: a splitter range [lo, hi] with lo == hi
    std::vector<uint32_t> single_list, single_of(nb, ~0u);
    for (uint32_t b = 0; b < nb; ++b) {
        const uint64_t lo = b ? hint.host[b - 1] : 0ull;
        const uint64_t hi = b + 1 < nb ? hint.host[b] - 1 : ~0ull;
        // worth pieces of its own when one workgroup would stream many chunks
        const bool big = !hint.share || hint.share[b] * (double)Bt > 4.0 * SINGLE_CHUNK;
        if (lo == hi && big) {
            single_of[b] = (uint32_t)single_list.size();
            single_list.push_back(b);
        }
    }
    n_single = (uint32_t)single_list.size();
    max_pieces = (uint32_t)((std::min(Bt, n) + SINGLE_CHUNK - 1) / SINGLE_CHUNK);
    UpPack up;
    const uint64_t o_cf = up.add(cf.data(), cf.size() * sizeof(Chunk));
    const uint64_t o_cl = up.add(cl.data(), cl.size() * sizeof(Chunk));
    const uint64_t o_slots = up.add(slots.data(), slots.size() * sizeof(FlatSlot));
    const uint64_t o_first = up.add(first, sizeof(first));
    const uint64_t o_dests = up.add(dests.data(), dests.size() * sizeof(Dest));
    const uint64_t o_sl = up.add(single_list.data(), single_list.size() * sizeof(uint32_t));
    const uint64_t o_so = up.add(single_of.data(), single_of.size() * sizeof(uint32_t));
    char* d = up.commit(E, A);
    d_single_list = n_single ? (uint32_t*)(d + o_sl) : nullptr;
    d_single_of = n_single ? (uint32_t*)(d + o_so) : nullptr;
    for (int z = 0; z < SETS; ++z)
        d_partials[z] = n_single ? A.take((uint64_t)n_single * max_pieces * single_partial_bytes()) : nullptr;
    d_chunks_full = (Chunk*)(d + o_cf);
    d_chunks_last = (Chunk*)(d + o_cl);
    d_slots = (FlatSlot*)(d + o_slots);
    d_first = (uint32_t*)(d + o_first);
    d_dests = (Dest*)(d + o_dests);
    d_regs = A.take_n<Region>(BP_CTL_RING);
    d_ctl = A.take_n<uint64_t>(BP_CTL_RING * ctl_words());
    scratch_off = A.off;
    const uint64_t hist = (uint64_t)nb * chunks_full;
    for (int z = 0; z < SETS; ++z) {
        part[z] = A.take_n<uint64_t>((Bt < n ? Bt : n) * (uint64_t)L.words);
        d_hist[z] = A.take_n<uint32_t>(hist + 1);
        d_offs[z] = A.take_n<uint64_t>(hist + 1);
    }
}

ColView BatchProgram::batch_src(uint64_t i) const {
    const uint64_t b0 = i * Bt;
    ColView v = src;
    v.key += b0;
    if (v.sum) v.sum += b0, v.mn += b0, v.mx += b0;
    if (v.fs) v.fs += b0;
    return v;
}

void BatchProgram::enqueue(Engine& E, uint64_t i, uint32_t slot, char* readback, hipStream_t st) {
    const uint64_t bn = batch_n(i);
    const bool last = i + 1 == batches;
    const Chunk* ch = last ? d_chunks_last : d_chunks_full;
    const uint32_t nch = last ? chunks_last : chunks_full;
    Region r;
    r.src = batch_src(i);
    r.n = bn;
    r.out_pos = 0;
    r.hist_base = 0;
    r.nb = nb;
    r.n_chunks = nch;
    Region* reg = d_regs + (i % BP_CTL_RING);
    uint64_t* ctl = d_ctl + (i % BP_CTL_RING) * ctl_words();
    const int z = (int)(i % SETS);
    E.pbegin("k_hist", st);
    launch_hist_batch(r, reg, ctl, (uint32_t)ctl_words(), ch, nch, splitters, d_hist[z], st);
    E.pend(bn, bn * 8, st);
    E.pbegin("k_scatter", st);
    launch_scatter(reg, ch, nch, splitters, d_offs[z], part[z], L, st, d_hist[z], d_offs[z], crow);
    E.pend(bn, bn * (uint64_t)L.words * 8, st);
    if (n_single) {
        E.pbegin("k_single_partial", st);
        launch_flat_single_partial(reg, d_offs[z], part[z], L, d_single_list, n_single, max_pieces, d_partials[z],
                                   st);
        E.pend(bn, 0, st);
    }
    E.pbegin("k_leaf", st);
    // the last leaf writes the control word and the group count straight to
    // the pinned readback slot (no copy after the launch)
    launch_leaf_flat(d_slots, nb, nullptr, reg, splitters, d_offs[z], part[z], L, d_first, d_dests + slot, ctl + 2,
                     ctl + 1, (uint32_t*)ctl, st, d_single_of, d_partials[z], max_pieces, E.ring_dev_of(readback));
    E.pend(bn, bn * (uint64_t)L.words * 8, st);
}

bool BatchProgram::result(const char* readback, uint64_t& groups) const {
    const uint64_t* h = (const uint64_t*)readback;
    const uint64_t err = h[0] >> 32;
    if (err & 1) throw Fail{ISA_EDEVICE, "leaf placement wait timed out"};
    if (err & 2) return false;
    groups = h[1];
    return true;
}

}  // namespace isa
