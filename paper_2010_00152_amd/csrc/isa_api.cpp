// C ABI of the grouping library (include/insort.h): argument checking, the
// run-generation loop with spilling, and the wide merge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "../../include/insort.h"
#include "isa_engine.h"

using namespace isa;

struct isa_ctx {
    int device = 0;
    int rungen = ISA_RUNGEN_READ_SORT_WRITE;
    // hybrid run generation: the resident index's share of the index memory
    uint32_t resident_permille = 800;
    // device address of the library-owned scratch on this context's device
    // (looked up at creation), used only by isa_group_by_noalloc
    void* scratch = nullptr;
    Engine eng;
    std::string last_error;
    std::mutex mu;
};

namespace {

void ck(hipError_t e, const char* what) {
    if (e != hipSuccess) throw Fail{ISA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool valid_aggs(uint32_t aggs) {
    return (aggs & ~(uint32_t)(ISA_COUNT | ISA_SUM_I64 | ISA_SUM_F64 | ISA_MIN_I64 | ISA_MAX_I64)) == 0;
}

Cols cols_of(uint32_t aggs) {
    Cols k;
    k.c = (aggs & ISA_COUNT) != 0;
    k.v = (aggs & (ISA_SUM_I64 | ISA_MIN_I64 | ISA_MAX_I64)) != 0;
    k.f = (aggs & ISA_SUM_F64) != 0;
    return k;
}

// Sort-reduce dispatch by size class: instances of at most FLAT_MAX rows take
// the flat plan (one partition level, no host round trip; optionally one
// graph launch); larger instances, or a flat attempt that met an oversized
// bucket, take the general multi-level plan.
std::vector<uint64_t> run_instances(Engine& E, Arena& A, const std::vector<Instance>& inst,
                                    const std::vector<Dest>& dests, const Cols& k, bool state_rows,
                                    const SplitterHint* hint, bool graph) {
    bool small = true;
    for (const Instance& x : inst) small &= x.n <= FLAT_MAX;
    if (small) {
        const uint64_t mark = A.off;
        std::vector<uint64_t> t;
        if (sort_reduce_flat(E, A, inst, dests, k, state_rows, hint, graph, t)) return t;
        A.off = mark;
    }
    return sort_reduce(E, A, inst, dests, k, state_rows, hint);
}

// Raw input rows viewed column-wise.
ColView input_view(const isa_input& in, const Cols& k) {
    ColView v;
    v.key = in.keys;
    v.cnt = nullptr;
    v.sum = v.mn = v.mx = k.v ? in.v_i64 : nullptr;
    v.fs = k.f ? in.v_f64 : nullptr;
    v.stride = 1;
    return v;
}

// Caller's output columns; unrequested columns are not written.
OutView output_view(const isa_output& o, uint32_t aggs, uint64_t shift) {
    OutView v;
    v.key = o.keys ? o.keys + shift : nullptr;
    v.cnt = (aggs & ISA_COUNT) && o.count ? o.count + shift : nullptr;
    v.sum = (aggs & ISA_SUM_I64) && o.sum_i64 ? o.sum_i64 + shift : nullptr;
    v.mn = (aggs & ISA_MIN_I64) && o.min_i64 ? o.min_i64 + shift : nullptr;
    v.mx = (aggs & ISA_MAX_I64) && o.max_i64 ? o.max_i64 + shift : nullptr;
    v.fs = (aggs & ISA_SUM_F64) && o.sum_f64 ? o.sum_f64 + shift : nullptr;
    v.stride = 1;
    return v;
}

isa_status check_output(const isa_output* out, uint32_t aggs, bool need_keys) {
    if (!out) return ISA_EINVAL;
    if (need_keys && !out->keys) return ISA_EINVAL;
    if ((aggs & ISA_COUNT) && !out->count) return ISA_EINVAL;
    if ((aggs & ISA_SUM_I64) && !out->sum_i64) return ISA_EINVAL;
    if ((aggs & ISA_SUM_F64) && !out->sum_f64) return ISA_EINVAL;
    if ((aggs & ISA_MIN_I64) && !out->min_i64) return ISA_EINVAL;
    if ((aggs & ISA_MAX_I64) && !out->max_i64) return ISA_EINVAL;
    return ISA_OK;
}

isa_status check_input(const isa_input* in, uint32_t aggs) {
    if (!in) return ISA_EINVAL;
    if (in->n_rows == 0) return ISA_OK;
    if (!in->keys) return ISA_EINVAL;
    if ((aggs & (ISA_SUM_I64 | ISA_MIN_I64 | ISA_MAX_I64)) && !in->v_i64) return ISA_EINVAL;
    if ((aggs & ISA_SUM_F64) && !in->v_f64) return ISA_EINVAL;
    return ISA_OK;
}

// ---------------------------------------------------------------------------
// Batch / capacity planning for run generation.
// ---------------------------------------------------------------------------

struct Plan {
    uint64_t batch_rows;  // Bt
    uint64_t capacity;    // K: rows the in-memory index may hold
};

constexpr uint64_t MIN_BATCH = 4 * (uint64_t)LEAF_CAP;
constexpr uint64_t MERGE_MARGIN = 2u << 20;

// Two merge control blocks of parts + 3 words, the splits (2 per part + 2)
// and the replacement-selection cursor.
uint64_t merge_scratch_bytes(uint64_t rows) {
    const uint64_t parts = merge_parts(rows, 0) + 2;
    return (4 * parts + 12) * 8 + 1024;
}

// Workspace used by run generation with batch Bt and index capacity K: two
// index buffers of K + Bt rows (the merge reads one and writes the other),
// three batch runs (one being sorted, one being absorbed, one kept until the
// previous absorb is decided), the merge's scratch, the batch program and the
// compact-run split's scratch.
// In-place absorption (read-sort-write): one index buffer of K + Bt rows
// absorbs each batch in place, and a spare area of a little over half of it
// receives a compacted run before its copy to host memory.
constexpr uint64_t SPARE_NUM = 11, SPARE_DEN = 20;
uint64_t spare_rows(uint64_t buf_rows) { return buf_rows * SPARE_NUM / SPARE_DEN + 64; }

uint64_t rungen_bytes(uint64_t Bt, uint64_t K, const Cols& k, bool inplace = false) {
    const uint64_t sw = (uint64_t)state_layout(k).words * 8;
    const uint64_t split_scratch = ((K + Bt) / 4096 + 4) * 48 + 1024;
    const uint64_t index = inplace ? ((K + Bt) + spare_rows(K + Bt)) * sw : 2 * (K + Bt) * sw;
    return index + 3 * Bt * sw + merge_scratch_bytes(K + 2 * Bt) + batch_program_bytes(Bt, k) + split_scratch +
           MERGE_MARGIN + 16 * 256 + (MAX_BUCKETS - 1) * 8;
}

// Share of the budget given to the batch area (1/share); the rest holds the
// index.  ISA_BATCH_SHARE overrides the default for tuning.
uint64_t batch_share() {
    const char* e = std::getenv("ISA_BATCH_SHARE");
    const long v = e ? std::atol(e) : 0;
    return v >= 2 && v <= 64 ? (uint64_t)v : 4;
}

bool plan_batches(uint64_t ws, uint64_t n, const Cols& k, Plan& p, bool inplace = false) {
    const uint64_t sw = (uint64_t)state_layout(k).words * 8;
    uint64_t Bt = ws / batch_share() / (sort_reduce_bytes(1, 0, k, false) - (4u << 20) + sw);
    // a batch is sorted by the flat plan
    Bt = std::min<uint64_t>(std::min<uint64_t>(Bt, n), FLAT_MAX);
    if (Bt < MIN_BATCH) Bt = MIN_BATCH;
    for (;;) {
        const uint64_t fixed = rungen_bytes(Bt, 0, k, inplace);
        if (fixed < ws) {
            // K from the remaining bytes: 2*K*sw (in place: about 1.55*K*sw)
            // plus merge scratch growth
            uint64_t K = (ws - fixed) / (2 * sw + 1);
            if (inplace) K = K * 2 * SPARE_DEN / (SPARE_DEN + SPARE_NUM);
            while (K > 0 && rungen_bytes(Bt, K, k, inplace) > ws) K -= std::max<uint64_t>(1, K / 64);
            // K >= 2 Bt: an index made of one batch always absorbs the next batch
            if (K >= 2 * Bt) {
                p.batch_rows = Bt;
                p.capacity = K;
                return true;
            }
        }
        if (Bt <= MIN_BATCH) return false;
        Bt = std::max<uint64_t>(MIN_BATCH, Bt / 2);
    }
}

// A run in the spill buffer: n_single count-1 rows stored column by column
// (single_bytes), then n_packed packed rows (packed_words), then n_multi rows
// in state layout, each part sorted on the key.  Runs written without count
// information hold only state rows (n_single = n_packed = 0).
struct RunInfo {
    uint64_t byte_off;
    uint64_t n_single;
    uint64_t n_multi;
    bool narrow = false;  // the count-1 part's integer values take 4 bytes
    uint64_t n_packed = 0;
};

// First row of [pos, n) whose key is >= x in a strided host array.
uint64_t lower_bound_strided(const uint64_t* keys, uint64_t stride, uint64_t pos, uint64_t n, uint64_t x) {
    uint64_t lo = pos, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (keys[mid * stride] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The wide merge (Section 4): every run and the in-memory index are consumed
// in one merge step, one key window at a time.  A window [start, end) is
// chosen so that the rows of all inputs inside it fit the staging area; the
// runs' "pages" are fence keys taken every P rows, and the next window ends at
// the largest fence whose window still fits (the forecasting order of page
// reads by the highest key read, Section 4 Figure 9).  Keys below the window
// end are final once the window is reduced; they are appended to the output.
//
// Runs are read in place from pinned host memory through its device mapping:
// one gather launch per window copies every slice into a staging buffer (and
// expands count-1 rows to state rows), on a side stream, two windows ahead of
// the window being reduced.  A window is cut at fence keys into pieces of at
// most PIECE_CAP rows; its pieces are reduced together by one flat launch
// sequence as key-ordered instances sharing the window's destination.
constexpr uint64_t PIECE_CAP = FLAT_MAX * 3 / 4;

// A preliminary merge step (Section 4, Example 4: steps that merge the
// smallest runs before a wide merge) writes its merged rows as one more run
// of state rows into the spill buffer, from byte `off` on, instead of into
// the caller's output.
struct RunSink {
    char* host = nullptr;  // the spill buffer (host address)
    uint64_t off = 0;      // where the run starts
    uint64_t cap = 0;      // bytes available from off
    uint64_t rows = 0;     // rows written
};

void wide_merge(Engine& E, Arena& A, const Cols& k, uint32_t aggs, const std::vector<RunInfo>& runs,
                const char* host, uint64_t* idx, uint64_t n_idx, isa_output* out, isa_stats* st,
                uint64_t& n_groups, RunSink* sink = nullptr) {
    const double t_enter = now_ms();
    const Layout S = state_layout(k);
    const Layout Rl = raw_layout(k);
    const uint64_t sw = (uint64_t)S.words;
    void* hdev = nullptr;
    if (hipHostGetDevicePointer(&hdev, (void*)host, 0) != hipSuccess || !hdev)
        throw Fail{ISA_EINVAL, "spill buffer is not device-mapped pinned memory"};
    const char* host_dev = (const char*)hdev;
    // Sources: every run contributes its count-1 sub-run (columns) and its
    // other rows (state rows); the last source is the index (state rows,
    // device).  keys: host view of the keys, strided; rows: device-visible
    // address of the rows (of the key column, for a count-1 sub-run).
    struct Src {
        const uint64_t* keys;
        uint64_t stride, n;
        const uint64_t* rows;
        bool raw, narrow;
        bool packed = false;
    };
    const uint64_t pw = (uint64_t)packed_words(S);
    std::vector<Src> src;
    auto on_dev = [&](const uint64_t* hp) { return (const uint64_t*)(host_dev + ((const char*)hp - host)); };
    uint64_t total = 0;
    for (const RunInfo& r : runs) {
        const uint64_t* base = (const uint64_t*)(host + r.byte_off);
        // the count-1 part is stored column by column, keys first
        if (r.n_single) src.push_back(Src{base, 1, r.n_single, on_dev(base), true, r.narrow});
        const uint64_t* pb = base + single_bytes(r.n_single, Rl, r.narrow) / 8;
        if (r.n_packed) src.push_back(Src{pb, pw, r.n_packed, on_dev(pb), false, false, true});
        const uint64_t* mb = pb + r.n_packed * pw;
        if (r.n_multi) src.push_back(Src{mb, sw, r.n_multi, on_dev(mb), false, false});
        total += r.n_single + r.n_packed + r.n_multi;
    }
    // the index's keys are read on the host from the pinned table (below)
    if (n_idx) src.push_back(Src{nullptr, 1, n_idx, idx, false, false});
    total += n_idx;
    const size_t ns = src.size();
    std::vector<uint64_t> pos(ns, 0);

    // window capacity W: three staging buffers (two windows gathered ahead of
    // the one being reduced), their gather task tables and the flat plan of a
    // window; a piece that falls back to the general plan is reduced alone
    const uint64_t avail0 = A.left() > (8u << 20) ? A.left() - (8u << 20) : 0;
    const uint64_t piece_fallback = sort_reduce_bytes(PIECE_CAP, 1, k, true);
    // gather tasks of one window: its pieces (at least PIECE_CAP/2 rows but
    // the last) each take one slice of every source, plus one per GATHER_ROWS
    auto win_task_bound = [&](uint64_t w) { return w / GATHER_ROWS + (ns + 1) * (w / (PIECE_CAP / 2) + 2) + 16; };
    auto need = [&](uint64_t w) {
        const uint64_t pieces = w / (PIECE_CAP / 2) + 2;
        return (sink ? 4 : 3) * w * sw * 8 +
               std::max(flat_bytes(w, pieces, k, true), std::min(piece_fallback, sort_reduce_bytes(w, 1, k, true)));
    };
    // every window but the last holds at least 3/4 W rows (fences every P rows)
    auto task_bound = [&](uint64_t w) { return (total / (w - w / 4) + 2) * win_task_bound(w); };
    uint64_t W = avail0 / ((sink ? 4 : 3) * sw * 8);
    while (W > 2 * (ns + 1) && need(W) > avail0) W -= W / 32 + 1;
    // ISA_FORCE_INDEX_SPILL=1 treats a merge beside an in-memory index as not
    // fitting (it lets tests reach the caller's fallback with ordinary inputs)
    const char* force = std::getenv("ISA_FORCE_INDEX_SPILL");
    if (W < 2 * (ns + 1) || need(W) > avail0 || (n_idx && force && force[0] == '1'))
        throw Fail{ISA_ESPILL, "workspace too small for a single wide merge of all runs"};
    // One pinned table holds the index's keys for the host's planning (a
    // kernel writes them there through the table's device mapping: no copy,
    // no staging) followed by the gather tasks of every window.
    const uint64_t max_tasks = task_bound(W);
    const uint64_t win_tasks = win_task_bound(W);
    const uint64_t keys_bytes = (n_idx * 8 + 255) & ~(uint64_t)255;
    char* h_table = (char*)E.table_buf(keys_bytes + (max_tasks + 1) * sizeof(GatherTask));
    char* h_table_dev = nullptr;
    ck(hipHostGetDevicePointer((void**)&h_table_dev, h_table, 0), "hipHostGetDevicePointer(task table)");
    if (n_idx) {
        launch_extract_keys(idx, n_idx, (uint32_t)sw, (uint64_t*)h_table_dev, E.stream);
        E.sync();
        src.back().keys = (const uint64_t*)h_table;
    }
    // Fences: the key of every P-th row of each source, merged in key order.
    // A cut at key x ends source s at lb_s(x) = its first row >= x; with c_s
    // of its fences below x, lb_s(x) lies in [c_s P, (c_s + 1) P], so the
    // fences bound the rows below x from above without touching the runs,
    // and one short search per source makes the chosen cut exact.
    const uint64_t P = std::max<uint64_t>(1, std::min(W, PIECE_CAP) / (4 * (ns + 1)));
    // The fences in key order come from a merge of the sources' fence
    // sequences (each source is sorted, so its fences are), produced only as
    // the sweep reaches them: the sweep for later windows runs while earlier
    // windows are being read.
    struct Fence {
        uint64_t key;
        uint32_t src;
    };
    std::vector<uint64_t> nf(ns), fnext(ns, 1);  // fences of a source: rows c*P for c = 1..nf
    uint64_t total_f = 0;
    for (size_t s = 0; s < ns; ++s) {
        nf[s] = src[s].n > P ? (src[s].n - 1) / P : 0;
        total_f += nf[s];
    }
    auto fkey = [&](size_t s, uint64_t c) { return src[s].keys[c * P * src[s].stride]; };
    using HeapEntry = std::pair<uint64_t, uint32_t>;
    std::priority_queue<HeapEntry, std::vector<HeapEntry>, std::greater<HeapEntry>> heap;
    for (size_t s = 0; s < ns; ++s)
        if (nf[s]) heap.push(HeapEntry{fkey(s, 1), (uint32_t)s});
    std::vector<Fence> fl;
    fl.reserve(total_f);
    auto F = [&](uint64_t j) -> const Fence& {  // j < total_f
        while (fl.size() <= j) {
            const HeapEntry h = heap.top();
            heap.pop();
            fl.push_back(Fence{h.first, h.second});
            if (++fnext[h.second] <= nf[h.second]) heap.push(HeapEntry{fkey(h.second, fnext[h.second]), h.second});
        }
        return fl[j];
    };
    std::vector<uint64_t> cnt(ns, 0);  // fences of each source below the last cut key
    uint64_t fi = 0;                   // first fence not below the last cut key
    auto hi_of = [&](size_t s, uint64_t c) { return std::min<uint64_t>(src[s].n, (c + 1) * P); };
    auto lb_in = [&](size_t s, uint64_t x) {
        const uint64_t lo = std::max<uint64_t>(pos[s], cnt[s] * P);
        return lower_bound_strided(src[s].keys, src[s].stride, lo, hi_of(s, cnt[s]), x);
    };
    // the next cut: all remaining rows if at most `cap`, else every row below
    // the largest fence key x whose bound on the rows below it is <= cap;
    // with no such key, the rows of the smallest key (at most one per source)
    // when `must`, else nothing
    auto next_cut = [&](uint64_t cap, bool must, std::vector<uint64_t>& end) -> uint64_t {
        uint64_t remaining = 0, min_key = ~0ull;
        for (size_t s = 0; s < ns; ++s) {
            remaining += src[s].n - pos[s];
            if (pos[s] < src[s].n) min_key = std::min(min_key, src[s].keys[pos[s] * src[s].stride]);
        }
        // (all remaining keys equal to the largest key value: at most one row per source)
        if (remaining <= cap || (must && min_key == ~0ull)) {
            for (size_t s = 0; s < ns; ++s) {
                end[s] = src[s].n;
                cnt[s] = nf[s];
            }
            fi = total_f;
            return remaining;
        }
        if (min_key == ~0ull) return 0;
        uint64_t U = 0;
        for (size_t s = 0; s < ns; ++s) U += hi_of(s, cnt[s]) - pos[s];
        uint64_t j = fi, best_j = total_f;
        uint64_t x = 0;
        while (j < total_f && U <= cap) {
            const uint64_t key = F(j).key;
            if (key > min_key) {
                x = key;
                best_j = j;
            }
            for (; j < total_f && F(j).key == key; ++j) {
                const uint32_t s = fl[j].src;
                U += hi_of(s, cnt[s] + 1) - hi_of(s, cnt[s]);
                ++cnt[s];
            }
        }
        if (best_j == total_f) {
            for (uint64_t t = fi; t < j; ++t) --cnt[fl[t].src];
            if (!must) return 0;
            x = min_key + 1;
            for (j = fi; j < total_f && F(j).key <= min_key; ++j) ++cnt[fl[j].src];
            best_j = j;
            // every fence at or below min_key is counted: each source's cut lies
            // in its bounded range
        } else {
            for (uint64_t t = best_j; t < j; ++t) --cnt[fl[t].src];
        }
        fi = best_j;
        uint64_t c = 0;
        for (size_t s = 0; s < ns; ++s) {
            end[s] = lb_in(s, x);
            c += end[s] - pos[s];
        }
        return c;
    };
    // Windows are planned one at a time, each just before its gather is
    // issued, so that the host plans while earlier windows are read.  A
    // window's gather tasks lay its pieces out one after the other in the
    // staging buffer; they are written to a pinned table (all windows, kept
    // for a second pass) that the gather reads through its device mapping.
    // (An upload of each window's tasks cost the host about 0.2 ms per
    // window in the runtime, which made the host loop the merge's
    // bottleneck.)
    GatherTask* h_tasks = (GatherTask*)(h_table + keys_bytes);
    GatherTask* const h_tasks_dev = (GatherTask*)(h_table_dev + keys_bytes);
    uint64_t n_tasks = 0;
    std::vector<uint64_t> task_first(1, 0);
    std::vector<uint64_t> win_rows, win_host_bytes;
    std::vector<std::vector<uint64_t>> win_pieces;
    std::vector<uint64_t> end(ns);
    uint64_t left = total;
    auto plan_next = [&]() -> bool {
        if (!left) return false;
        uint64_t at = 0, hb = 0;
        std::vector<uint64_t> pieces;
        while (left && at < W) {
            const uint64_t c = next_cut(std::min(PIECE_CAP, W - at), at == 0, end);
            if (c == 0) break;  // the next piece would not fit this window
            for (size_t s = 0; s < ns; ++s) {
                const Src& q = src[s];
                // host bytes per row; a count-1 part's columns
                const uint64_t row_bytes = q.raw      ? 8 + (Rl.fs >= 0 ? 8 : 0) + (Rl.sum >= 0 ? (q.narrow ? 4 : 8) : 0)
                                           : q.packed ? pw * 8
                                                      : sw * 8;
                const uint64_t* fs_c = q.rows + q.n;
                const uint64_t* int_c = q.rows + q.n * (Rl.fs >= 0 ? 2 : 1);
                for (uint64_t r = pos[s]; r < end[s]; r += GATHER_ROWS) {
                    const uint64_t len = std::min<uint64_t>(GATHER_ROWS, end[s] - r);
                    if (n_tasks >= max_tasks || n_tasks - task_first.back() >= win_tasks)
                        throw Fail{ISA_EDEVICE, "internal: gather task table overflow"};
                    GatherTask& t = h_tasks[n_tasks++];
                    t.dst_row = at;
                    t.n = (uint32_t)len;
                    if (q.raw) {
                        t.src = q.rows + r;
                        t.fv = Rl.fs >= 0 ? fs_c + r : nullptr;
                        t.iv = Rl.sum < 0 ? nullptr
                               : q.narrow ? (const void*)((const int32_t*)int_c + r)
                                          : (const void*)(int_c + r);
                        t.raw = q.narrow ? 2u : 1u;
                    } else {
                        t.src = q.rows + r * (q.packed ? pw : sw);
                        t.fv = nullptr;
                        t.iv = nullptr;
                        t.raw = q.packed ? 3u : 0u;
                    }
                    at += len;
                    if (s + 1 < ns || !n_idx) hb += len * row_bytes;
                }
            }
            pieces.push_back(c);
            left -= c;
            pos = end;
        }
        win_rows.push_back(at);
        win_host_bytes.push_back(hb);
        win_pieces.push_back(pieces);
        task_first.push_back(n_tasks);
        return true;
    };
    size_t planned = 0;
    auto have = [&](size_t w) {
        while (planned <= w && plan_next()) ++planned;
        return w < planned;
    };
    uint64_t* stage[3];
    for (int j = 0; j < 3; ++j) stage[j] = A.take_n<uint64_t>(W * sw);
    uint64_t* sink_rows = sink ? A.take_n<uint64_t>(W * sw) : nullptr;
    // output cursors on the device: window w starts at the end row that
    // window w-1 wrote (cur[(w+1) % 2]) and writes its own end to cur[w % 2]
    uint64_t* d_cur = A.take_n<uint64_t>(2);
    const uint64_t mark = A.off;
    hipStream_t gs = E.side(0);
    auto ev_gather = [&](size_t w) { return E.sync_event(5 + (w % 3)); };
    auto ev_reduce = [&](size_t w) { return E.sync_event(12 + (w % 3)); };
    auto issue = [&](size_t w) {
        const uint64_t t0 = task_first[w], nt = task_first[w + 1] - task_first[w];
        E.pbegin("merge_h2d", gs);
        launch_gather(h_tasks_dev + t0, (uint32_t)nt, Rl, S, stage[w % 3], gs);
        E.pend(win_rows[w], win_host_bytes[w], gs);
        ck(hipEventRecord(ev_gather(w), gs), "hipEventRecord");
    };
    auto pieces_of = [&](size_t w) {
        std::vector<Instance> inst;
        uint64_t row = 0;
        for (uint64_t pc : win_pieces[w]) {
            Instance x;
            x.src = aos_view(stage[w % 3] + row * sw, S);
            x.n = pc;
            x.dest = 0;
            inst.push_back(x);
            row += pc;
        }
        return inst;
    };
    // the gathers follow everything enqueued on the caller's stream so far
    launch_fill(d_cur, 2, 0, E.stream);
    ck(hipEventRecord(E.sync_event(4), E.stream), "hipEventRecord");
    ck(hipStreamWaitEvent(gs, E.sync_event(4), 0), "hipStreamWaitEvent");

    if (sink) {
        // A preliminary merge step: windows one at a time, each reduced into
        // a device buffer whose rows are then appended to the new run in the
        // spill buffer.
        for (size_t w = 0; w < 2 && have(w); ++w) issue(w);
        for (size_t w = 0; have(w); ++w) {
            if (have(w + 2)) {
                if (w >= 1) ck(hipStreamWaitEvent(gs, ev_reduce(w - 1), 0), "hipStreamWaitEvent");
                issue(w + 2);
            }
            ck(hipStreamWaitEvent(E.stream, ev_gather(w), 0), "hipStreamWaitEvent");
            A.off = mark;
            Dest d;
            d.out = aos_out(sink_rows, S);
            d.capacity = W;
            const std::vector<Instance> inst = pieces_of(w);
            uint64_t g = 0;
            std::vector<uint64_t> gv;
            if (sort_reduce_flat(E, A, inst, std::vector<Dest>(1, d), k, true, nullptr, false, gv)) {
                g = gv[0];
            } else {
                for (const Instance& x : inst) {
                    A.off = mark;
                    Dest dx = d;
                    dx.out = aos_out(sink_rows + g * sw, S);
                    dx.capacity = W - g;
                    g += sort_reduce(E, A, std::vector<Instance>(1, x), std::vector<Dest>(1, dx), k, true)[0];
                }
            }
            ck(hipEventRecord(ev_reduce(w), E.stream), "hipEventRecord");
            const uint64_t bytes = g * sw * 8;
            if ((sink->rows * sw * 8) + bytes > sink->cap) throw Fail{ISA_ESPILL, "spill buffer too small"};
            if (g) {
                E.pbegin("merge_d2h");
                ck(hipMemcpyAsync(sink->host + sink->off + sink->rows * sw * 8, sink_rows, bytes,
                                  hipMemcpyDeviceToHost, E.stream),
                   "hipMemcpyAsync(merged run)");
                E.pend(g, bytes);
            }
            E.sync();  // the device buffer is reused by the next window
            sink->rows += g;
        }
        ck(hipStreamSynchronize(gs), "hipStreamSynchronize(gather)");
        A.off = mark;
        n_groups = sink->rows;
        return;
    }
    // First pass, without host round trips: every window's reduction is
    // enqueued behind its gather and places its groups after the device-side
    // cursor of the window before; a gather into stage[w % 3] waits for the
    // reduction of window w-3, the buffer's last reader.
    for (size_t w = 0; w < 2 && have(w); ++w) issue(w);
    if (st) st->t_plan_ms = now_ms() - t_enter;
    std::vector<const uint64_t*> win_ctl;
    size_t nw = 0;
    for (size_t w = 0; have(w); ++w) {
        if (have(w + 2)) {
            if (w >= 1) ck(hipStreamWaitEvent(gs, ev_reduce(w - 1), 0), "hipStreamWaitEvent");
            issue(w + 2);
        }
        ck(hipStreamWaitEvent(E.stream, ev_gather(w), 0), "hipStreamWaitEvent");
        A.off = mark;
        Dest d;
        d.out = output_view(*out, aggs, 0);
        d.capacity = out->capacity;
        d.base = d_cur + ((w + 1) % 2);
        std::vector<uint64_t> g;
        const uint64_t* hc = nullptr;
        sort_reduce_flat(E, A, pieces_of(w), std::vector<Dest>(1, d), k, true, nullptr, false, g, d_cur + (w % 2),
                         &hc);
        if (!hc) throw Fail{ISA_EDEVICE, "internal: empty wide-merge window"};
        win_ctl.push_back(hc);
        ck(hipEventRecord(ev_reduce(w), E.stream), "hipEventRecord");
        nw = w + 1;
    }
    const uint64_t* h_end = (const uint64_t*)download_async(E, d_cur + ((nw + 1) % 2), 8);
    ck(hipStreamSynchronize(gs), "hipStreamSynchronize(gather)");
    ck(hipStreamSynchronize(E.stream), "hipStreamSynchronize");
    bool redo = false;
    for (const uint64_t* hc : win_ctl) {
        const uint64_t err = hc[0] >> 32;
        if (err & 1) throw Fail{ISA_EDEVICE, "leaf placement wait timed out"};
        redo |= (err & 2) != 0;
    }
    uint64_t cursor = *h_end;
    E.sync();
    if (st) st->windows += nw;
    // ISA_FORCE_MERGE_REDO=1 takes the second pass as if a window had failed
    // (it lets tests reach that path with ordinary inputs)
    if (const char* f = std::getenv("ISA_FORCE_MERGE_REDO")) redo |= f[0] == '1';
    if (redo) {
        // A window held a bucket too large for a leaf, so the placement of
        // the windows after it is void.  Second pass, one window at a time
        // with the output cursor on the host; a window whose flat plan fails
        // reduces its pieces one at a time with the general plan.
        cursor = 0;
        for (size_t w = 0; w < 2 && w < nw; ++w) issue(w);
        for (size_t w = 0; w < nw; ++w) {
            if (w + 2 < nw) issue(w + 2);
            ck(hipStreamWaitEvent(E.stream, ev_gather(w), 0), "hipStreamWaitEvent");
            A.off = mark;
            auto dest_at = [&](uint64_t c) {
                Dest dd;
                dd.out = output_view(*out, aggs, std::min(c, out->capacity));
                dd.capacity = out->capacity > c ? out->capacity - c : 0;
                return dd;
            };
            const std::vector<Instance> inst = pieces_of(w);
            std::vector<uint64_t> g;
            if (sort_reduce_flat(E, A, inst, std::vector<Dest>(1, dest_at(cursor)), k, true, nullptr, false, g)) {
                cursor += g[0];
            } else {
                for (const Instance& x : inst) {
                    A.off = mark;
                    cursor += sort_reduce(E, A, std::vector<Instance>(1, x), std::vector<Dest>(1, dest_at(cursor)),
                                          k, true)[0];
                }
            }
            ck(hipEventRecord(ev_reduce(w), E.stream), "hipEventRecord");
        }
        ck(hipStreamSynchronize(gs), "hipStreamSynchronize(gather)");
    }
    A.off = mark;
    n_groups = cursor;
}

isa_status fail(isa_ctx* ctx, const Fail& f) {
    if (ctx) {
        ctx->eng.drain();
        ctx->last_error = f.what;
    }
    return (isa_status)f.status;
}

}  // namespace

extern "C" {

const char* isa_status_str(isa_status st) {
    switch (st) {
        case ISA_OK: return "ok";
        case ISA_EINVAL: return "invalid argument";
        case ISA_EBUDGET: return "workspace below the minimum";
        case ISA_ESPILL: return "spill buffer too small or too many runs";
        case ISA_ETRUNC: return "output capacity below the group count";
        case ISA_EDEVICE: return "HIP device error";
        case ISA_ENOMEM: return "out of memory";
        case ISA_EUNIMPL: return "not implemented";
        case ISA_EBUSY: return "busy";
    }
    return "unknown status";
}

const char* isa_last_error(isa_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

isa_status isa_ctx_create(int device, isa_ctx** out) {
    if (!out) return ISA_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return ISA_EDEVICE;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return ISA_EDEVICE;
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) return ISA_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return ISA_EDEVICE;
    isa_ctx* c = new (std::nothrow) isa_ctx();
    if (!c) return ISA_ENOMEM;
    c->device = device;
    c->eng.device = device;
    // set-up for the entry point that must not allocate: the scratch's address
    // on this device, and the host-side staging it uses
    if (noalloc_scratch(device, &c->scratch) != hipSuccess || !c->scratch) {
        delete c;
        return ISA_EDEVICE;
    }
    try {
        c->eng.prepare_no_alloc();
    } catch (const Fail& f) {
        c->eng.release();
        delete c;
        return (isa_status)f.status;
    }
    *out = c;
    return ISA_OK;
}

void isa_ctx_destroy(isa_ctx* ctx) {
    if (!ctx) return;
    ctx->eng.release();
    delete ctx;
}

isa_status isa_profile_enable(isa_ctx* ctx, int on) {
    if (!ctx) return ISA_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->eng.prof_on = on != 0;
    ctx->eng.prof.clear();
    ctx->eng.ev_used = 0;
    return ISA_OK;
}

int isa_profile_read(isa_ctx* ctx, isa_kernel_time* out, int max) {
    if (!ctx) return ISA_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    std::vector<isa_kernel_time> agg;
    for (const ProfRec& r : ctx->eng.prof) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            return ISA_EDEVICE;
        size_t i = 0;
        while (i < agg.size() && std::strncmp(agg[i].name, r.name, sizeof(agg[i].name)) != 0) ++i;
        if (i == agg.size()) {
            isa_kernel_time t;
            std::memset(&t, 0, sizeof(t));
            std::strncpy(t.name, r.name, sizeof(t.name) - 1);
            agg.push_back(t);
        }
        agg[i].launches += 1;
        agg[i].rows += r.rows;
        agg[i].bytes += r.bytes;
        agg[i].total_ms += ms;
    }
    const int n = (int)agg.size() < max ? (int)agg.size() : max;
    for (int i = 0; i < n; ++i) out[i] = agg[i];
    return (int)agg.size();
}

uint64_t isa_state_row_bytes(uint32_t aggs) { return (uint64_t)state_layout(cols_of(aggs)).words * 8; }

uint64_t isa_min_workspace_bytes(uint32_t aggs) {
    const Cols k = cols_of(aggs);
    return rungen_bytes(MIN_BATCH, 2 * MIN_BATCH, k);
}

uint64_t isa_noalloc_max_rows(uint32_t aggs) {
    if (!valid_aggs(aggs)) return 0;
    const Cols k = cols_of(aggs);
    uint64_t lo = 0, hi = NOALLOC_SCRATCH_BYTES;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) / 2;
        if (sort_reduce_bytes(mid, 1, k, false) <= NOALLOC_SCRATCH_BYTES) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

isa_status isa_group_by_noalloc(isa_ctx* ctx, const isa_input* in, uint32_t aggs, isa_output* out, void* stream) {
    if (out) out->n_groups = 0;
    if (!ctx || !valid_aggs(aggs)) return ISA_EINVAL;
    isa_status s = check_input(in, aggs);
    if (s != ISA_OK) return s;
    s = check_output(out, aggs, true);
    if (s != ISA_OK) return s;
    if (in->n_rows == 0) return ISA_OK;
    if (in->n_rows > isa_noalloc_max_rows(aggs)) return ISA_EBUDGET;
    if (!ctx->scratch) return ISA_EDEVICE;
    std::lock_guard<std::mutex> lock(ctx->mu);
    Engine& E = ctx->eng;
    struct NoAlloc {  // the engine refuses to allocate until the call returns
        Engine& e;
        explicit NoAlloc(Engine& x) : e(x) { e.no_alloc = true; }
        ~NoAlloc() { e.no_alloc = false; }
    } guard(E);
    try {
        ck(hipSetDevice(ctx->device), "hipSetDevice");
        E.stream = (hipStream_t)stream;
        const Cols k = cols_of(aggs);
        // the scratch takes the place of the workspace; nothing in it needs
        // to start at zero (every buffer a plan reads is written or cleared
        // by that plan's own launches on this stream)
        Arena A;
        A.base = (char*)ctx->scratch;
        A.cap = NOALLOC_SCRATCH_BYTES;
        Dest d;
        d.out = output_view(*out, aggs, 0);
        d.capacity = out->capacity;
        std::vector<Instance> inst(1);
        inst[0].src = input_view(*in, k);
        inst[0].n = in->n_rows;
        inst[0].dest = 0;
        const uint64_t g = run_instances(E, A, inst, std::vector<Dest>(1, d), k, false, nullptr, false)[0];
        E.sync();
        out->n_groups = g;
        return g > out->capacity ? ISA_ETRUNC : ISA_OK;
    } catch (const Fail& f) {
        out->n_groups = 0;
        return fail(ctx, f);
    } catch (const std::bad_alloc&) {
        out->n_groups = 0;
        return ISA_ENOMEM;
    }
}

isa_status isa_group_by(isa_ctx* ctx, const isa_input* in, uint32_t aggs, isa_workspace ws, isa_spill spill,
                        isa_output* out, isa_stats* stats, void* stream) {
    if (out) out->n_groups = 0;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!ctx || !valid_aggs(aggs)) return ISA_EINVAL;
    isa_status s = check_input(in, aggs);
    if (s != ISA_OK) return s;
    s = check_output(out, aggs, true);
    if (s != ISA_OK) return s;
    if (in->n_rows == 0) return ISA_OK;
    if (!ws.dev || ((uintptr_t)ws.dev & 255)) return ISA_EINVAL;
    const Cols k = cols_of(aggs);
    if (ws.bytes < isa_min_workspace_bytes(aggs)) return ISA_EBUDGET;
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        ck(hipSetDevice(ctx->device), "hipSetDevice");
        Engine& E = ctx->eng;
        E.stream = (hipStream_t)stream;
        Arena A;
        A.base = (char*)ws.dev;
        A.cap = ws.bytes;
        const double t0 = now_ms();
        const uint64_t n = in->n_rows;
        const Layout S = state_layout(k);
        const uint64_t sw = (uint64_t)S.words;
        const ColView src = input_view(*in, k);
        uint64_t n_groups = 0;

        if (sort_reduce_bytes(n, 1, k, false) <= ws.bytes) {
            // The output fits memory and the whole input is one batch: the
            // index never fills, no run is written (Section 5: no spilling
            // when the output fits memory).
            Dest d;
            d.out = output_view(*out, aggs, 0);
            d.capacity = out->capacity;
            std::vector<Instance> inst(1);
            inst[0].src = src;
            inst[0].n = n;
            inst[0].dest = 0;
            n_groups = run_instances(E, A, inst, std::vector<Dest>(1, d), k, false, nullptr, false)[0];
            if (stats) {
                stats->batches = 1;
                stats->batch_rows = n;
                stats->index_capacity = n;
                stats->peak_ws_bytes = A.peak;
                stats->t_rungen_ms = now_ms() - t0;
            }
        } else {
            Plan p;
            const bool rs = ctx->rungen == ISA_RUNGEN_REPLACEMENT;
            const bool hy = ctx->rungen == ISA_RUNGEN_HYBRID;
            // compact runs need a count column and a raw row narrower than a state row
            const Layout Rl = raw_layout(k);
            const bool compact = S.cnt >= 0 && Rl.words < S.words;
            // read-sort-write absorbs every batch into one index buffer in
            // place when a compacted run of mostly count-1 rows fits a spare
            // area of about half the index (a raw row at most half a state
            // row); replacement selection and hybrid run generation keep the
            // old index while the merged one is decided (two buffers)
            const bool inplace = !rs && !hy && compact && 2 * Rl.words <= S.words;
            if (!plan_batches(ws.bytes, n, k, p, inplace)) return ISA_EBUDGET;
            // Hybrid run generation: the index memory is shared by a resident
            // index (Kr keys) and a run-generation index (Kw keys, at least a
            // batch), and runs are compacted in a staging area of their own
            // (a run-generation index and a demotion at most).
            uint64_t Kr = 0, Kw = 0, st_rows = 0;
            if (hy) {
                // plan with the staging area set aside, until the plan and
                // its staging area fit together
                const uint64_t swb = (uint64_t)S.words * 8;
                uint64_t stage_bytes = 0;
                bool fits = false;
                for (int it = 0; it < 16 && !fits; ++it) {
                    if (stage_bytes >= ws.bytes || !plan_batches(ws.bytes - stage_bytes, n, k, p)) return ISA_EBUDGET;
                    Kw = std::max<uint64_t>(p.batch_rows, p.capacity * (1000 - ctx->resident_permille) / 1000);
                    Kr = p.capacity > Kw ? p.capacity - Kw : 0;
                    // a resident index smaller than a batch is no resident index
                    if (Kr < p.batch_rows) Kr = 0;
                    st_rows = Kr / 4 + Kw + p.batch_rows;
                    const uint64_t need = st_rows * swb + 4096;
                    fits = rungen_bytes(p.batch_rows, p.capacity, k) + need <= ws.bytes;
                    stage_bytes = std::max(need, stage_bytes + stage_bytes / 8 + 4096);
                }
                if (!fits) return ISA_EBUDGET;
            }
            const uint64_t buf_rows = p.capacity + p.batch_rows;
            const uint64_t buf_bytes = buf_rows * sw * 8;
            uint64_t* idx[2];
            idx[0] = A.take_n<uint64_t>(buf_rows * sw);
            idx[1] = inplace ? nullptr : A.take_n<uint64_t>(buf_rows * sw);
            // in place: the area a compacted run is written to before its copy
            const uint64_t spare_words = inplace ? spare_rows(buf_rows) * sw : 0;
            uint64_t* spare = inplace ? A.take_n<uint64_t>(spare_words) : nullptr;
            uint64_t* brun[3];
            for (int j = 0; j < 3; ++j) brun[j] = A.take_n<uint64_t>(p.batch_rows * sw);
            const uint64_t mscr_parts = merge_parts(buf_rows, p.batch_rows) + 1;
            // merge control block: [ticket, error], merged row count, the
            // replacement-selection cursor's row, per-partition status; then
            // the partition splits
            // two control blocks, used by alternate merges; each merge clears
            // the other one for the next merge
            const uint64_t mctl_words = mscr_parts + 3;
            uint64_t* m_ctl2[2];
            m_ctl2[0] = A.take_n<uint64_t>(2 * mctl_words);
            m_ctl2[1] = m_ctl2[0] + mctl_words;
            launch_fill(m_ctl2[0], 2 * mctl_words, 0, E.stream);
            // replacement selection: the cursor key and its past-the-end flag
            uint64_t* rs_cur = A.take_n<uint64_t>(2);
            launch_fill(rs_cur, 2, 0, E.stream);
            // hybrid: the cut below which keys stay resident, in the same two
            // words (key, above-every-key flag); it starts above every key
            if (hy && Kr) launch_fill(rs_cur + 1, 1, 1, E.stream);
            uint64_t* m_splits = A.take_n<uint64_t>(2 * (mscr_parts + 1));
            uint64_t* hy_stage = hy ? A.take_n<uint64_t>(st_rows * sw) : nullptr;
            const uint64_t sp_blocks = split_blocks(buf_rows) + 1;
            uint32_t* sp_counts = A.take_n<uint32_t>(2 * sp_blocks);
            uint64_t* sp_offs = A.take_n<uint64_t>(2 * sp_blocks + 4);
            uint64_t* sp_tiles = A.take_n<uint64_t>(scan_tiles(sp_blocks) + 1);
            // splitters for every batch, chosen once from a sample of the whole
            // input (batches are slices of one input)
            uint64_t* d_gspl = A.take_n<uint64_t>(MAX_BUCKETS - 1);
            std::vector<uint64_t> h_gspl;
            std::vector<double> share;
            double light_share = 0;
            const uint32_t nb_batch = buckets_for(E, p.batch_rows);
            choose_splitters(E, A, src, n, nb_batch, d_gspl, h_gspl, &share, &light_share);
            // heavy keys take buckets of their own; the largest bucket that
            // spans several keys must stay well below a leaf, so skew that
            // crowds the light keys into fewer buckets shortens the batches
            if (light_share > 0) {
                const double lim = 0.6 * LEAF_CAP / light_share;
                if (lim < (double)p.batch_rows) p.batch_rows = std::max<uint64_t>(MIN_BATCH, (uint64_t)lim);
            }
            SplitterHint hint;
            hint.dev = d_gspl;
            hint.host = h_gspl.data();
            hint.nb = nb_batch;
            hint.share = share.data();
            std::vector<Dest> bdest(3);
            for (int j = 0; j < 3; ++j) {
                bdest[j].out = aos_out(brun[j], S);
                bdest[j].capacity = p.batch_rows;
            }
            BatchProgram bp;
            bp.setup(E, A, src, n, p.batch_rows, k, hint, bdest);
            const uint64_t top = A.off;

            // The batches form a software pipeline on the stream: batch i+1 is
            // sorted while the host decides on the absorb of batch i-1, so the
            // device never waits for a host round trip.  Batch runs rotate over
            // three buffers.
            // The index is `ip` (n_idx rows): one of the two index buffers, or,
            // right after a spill or at the first batch, the batch run that
            // starts it (K >= 2 Bt guarantees that the next merge absorbs it,
            // before its buffer is reused).  In place, the index lies at the
            // head of the one index buffer or at its tail (ending at row
            // buf_rows), and is empty (ip null) after a spill.
            const uint64_t* ip = nullptr;
            uint64_t n_idx = 0;
            std::vector<RunInfo> runs;
            uint64_t spill_used = 0, spilled_bytes = 0;  // bytes of the spill buffer in use
            uint64_t batches = 0, spilled = 0;
            // a run still being copied to host memory occupies idx[pend_buf]
            // from byte pend_lo to its end
            int pend_buf = -1;
            uint64_t pend_lo = 0;
            // in place: a run is being copied to host memory from the index
            // buffer itself (pend_idx), or from the spare area (spare_busy)
            bool pend_idx = false, spare_busy = false;
            hipStream_t cs = E.copier();
            // runs are written to the pinned spill buffer through its device mapping
            char* spill_dev = nullptr;
            if (spill.host_pinned) {
                void* p_dev = nullptr;
                if (hipHostGetDevicePointer(&p_dev, spill.host_pinned, 0) != hipSuccess || !p_dev)
                    throw Fail{ISA_EINVAL, "spill buffer is not device-mapped pinned memory"};
                spill_dev = (char*)p_dev;
            }
            auto ev_sort = [&](uint64_t i) { return E.sync_event(16 + (i % 4)); };
            auto ev_merge = [&](uint64_t i) { return E.sync_event(20 + (i % 4)); };
            auto rb_sort = [&](uint64_t i) { return E.ring_slot(i % 8); };
            auto rb_merge = [&](uint64_t i) { return E.ring_slot(8 + (i % 8)); };
            // the index buffer the next merge writes: not the index itself, and
            // preferably not the one whose tail holds a run being copied out
            auto merge_target = [&]() -> int {
                if (inplace) return 0;
                if (ip == idx[0]) return 1;
                if (ip == idx[1]) return 0;
                return pend_buf == 0 ? 1 : 0;
            };
            // a compact run whose size the host has not read yet: its copy to
            // host memory is enqueued by flush_copy once the split count is in
            struct {
                bool active = false;
                int buf = 0;
                const uint64_t* src = nullptr;  // in place: the run's state rows
                uint64_t rows = 0;
            } deferred;
            auto flush_copy = [&]() {
                if (!deferred.active) return;
                deferred.active = false;
                ck(hipEventSynchronize(E.sync_event(2)), "hipEventSynchronize(split count)");
                const uint64_t n_run = deferred.rows;
                uint64_t n_single = ((const uint64_t*)E.ring_slot(16))[0];
                bool narrow = ((const uint64_t*)E.ring_slot(16))[1] != 0;
                uint64_t n_packed = ((const uint64_t*)E.ring_slot(16))[2];
                uint64_t bytes = compact_bytes(n_single, n_packed, n_run - n_single - n_packed, Rl, S, narrow);
                const char* run_src = inplace ? (const char*)spare : (const char*)idx[deferred.buf] + buf_bytes - bytes;
                if (inplace && bytes / 8 > spare_words) {
                    // the split wrote nothing (the compacted run exceeds the
                    // spare area): the run's state rows go out as they are, and
                    // the index buffer stays read until the copy ends
                    n_single = 0;
                    n_packed = 0;
                    narrow = false;
                    bytes = n_run * sw * 8;
                    run_src = (const char*)deferred.src;
                    pend_idx = true;
                } else if (inplace) {
                    spare_busy = true;
                }
                if (spill_used + bytes > spill.bytes) throw Fail{ISA_ESPILL, "spill buffer too small"};
                ck(hipStreamWaitEvent(cs, E.sync_event(2), 0), "hipStreamWaitEvent");
                E.pbegin("spill_d2h", cs);
                ck(hipMemcpyAsync(spill_dev + spill_used, run_src, bytes, hipMemcpyDeviceToDeviceNoCU, cs),
                   "hipMemcpyAsync(spill)");
                E.pend(n_run, bytes, cs);
                ck(hipEventRecord(E.sync_event(1), cs), "hipEventRecord");
                RunInfo ri;
                ri.byte_off = spill_used;
                ri.n_single = n_single;
                ri.n_packed = n_packed;
                ri.n_multi = n_run - n_single - n_packed;
                ri.narrow = narrow;
                runs.push_back(ri);
                spill_used += bytes;
                spilled += n_run;
                spilled_bytes += bytes;
                if (!inplace) pend_lo = buf_bytes - bytes;
            };
            // in place: order the stream after a copy that reads the index buffer
            auto guard_idx = [&]() {
                flush_copy();
                if (pend_idx) {
                    ck(hipStreamWaitEvent(E.stream, E.sync_event(1), 0), "hipStreamWaitEvent");
                    pend_idx = false;
                }
            };
            // order the stream after the pending run's copy when [0, end) of
            // idx[buf] is about to be written over it
            auto guard = [&](int buf, uint64_t end) {
                if (pend_buf == buf) flush_copy();
                if (pend_buf == buf && end > pend_lo) {
                    ck(hipStreamWaitEvent(E.stream, E.sync_event(1), 0), "hipStreamWaitEvent");
                    pend_buf = -1;
                }
            };
            // memory is full: write the index as one sorted run (read-sort-write).
            // The run is split into its count-1 rows (raw layout) and the others,
            // placed at the end of the other index buffer, and copied to host
            // memory on the copy stream while run generation continues.  The
            // copy's size depends on the split's count, so the copy is enqueued
            // later (flush_copy: once the next batch has started the next
            // index), when the count is in.
            auto spill_index = [&]() {
                flush_copy();
                // an index that fails to absorb a batch holds more than one
                // batch, so it lives in an index buffer
                if (ip != idx[0] && ip != idx[1]) throw Fail{ISA_EDEVICE, "internal: spilling a batch run"};
                if (!spill.host_pinned) throw Fail{ISA_ESPILL, "spill buffer too small"};
                const int own = ip == idx[0] ? 0 : 1;
                const int spare = own ^ 1;
                if (pend_buf >= 0) {
                    ck(hipStreamWaitEvent(E.stream, E.sync_event(1), 0), "hipStreamWaitEvent");
                    pend_buf = -1;
                }
                if (compact) {
                    launch_split(ip, n_idx, S, Rl, sp_counts, sp_tiles, sp_offs, idx[spare], buf_rows * sw, E.stream);
                    // the count-1 rows and the narrow flag
                    ck(hipMemcpyAsync(E.ring_slot(16), sp_offs + split_blocks(n_idx), 24, hipMemcpyDeviceToHost,
                                      E.stream),
                       "hipMemcpyAsync(split count)");
                    ck(hipEventRecord(E.sync_event(2), E.stream), "hipEventRecord");
                    deferred.active = true;
                    deferred.buf = spare;
                    deferred.rows = n_idx;
                    // the whole spare buffer counts as in use until the size is known
                    pend_buf = spare;
                    pend_lo = 0;
                    n_idx = 0;
                    return;
                }
                const uint64_t bytes = n_idx * sw * 8;
                if (spill_used + bytes > spill.bytes) throw Fail{ISA_ESPILL, "spill buffer too small"};
                ck(hipEventRecord(E.sync_event(0), E.stream), "hipEventRecord");
                ck(hipStreamWaitEvent(cs, E.sync_event(0), 0), "hipStreamWaitEvent");
                // one runtime copy on the copy stream: a kernel of our own
                // writing host memory slows the concurrent kernels far more
                E.pbegin("spill_d2h", cs);
                ck(hipMemcpyAsync(spill_dev + spill_used, ip, bytes, hipMemcpyDeviceToDeviceNoCU, cs),
                   "hipMemcpyAsync(spill)");
                E.pend(n_idx, bytes, cs);
                ck(hipEventRecord(E.sync_event(1), cs), "hipEventRecord");
                RunInfo ri;
                ri.byte_off = spill_used;
                ri.n_single = 0;
                ri.n_multi = n_idx;
                runs.push_back(ri);
                spill_used += bytes;
                spilled += n_idx;
                spilled_bytes += bytes;
                pend_buf = own;
                pend_lo = 0;
                n_idx = 0;
            };
            // memory is full, in place: the merged index U (m rows, more than
            // K) is written whole as one run, and the next index starts with
            // the next batch run.  The run is compacted into the spare area
            // (after the spare area's last copy) and copied to host memory by
            // flush_copy; a compacted run larger than the spare area is not
            // written there, and flush_copy copies U's state rows instead.
            auto spill_inplace = [&](const uint64_t* U, uint64_t m) {
                flush_copy();
                if (!spill.host_pinned) throw Fail{ISA_ESPILL, "spill buffer too small"};
                if (spare_busy) {
                    ck(hipStreamWaitEvent(E.stream, E.sync_event(1), 0), "hipStreamWaitEvent");
                    spare_busy = false;
                }
                launch_split(U, m, S, Rl, sp_counts, sp_tiles, sp_offs, spare, 0, E.stream, spare_words);
                ck(hipMemcpyAsync(E.ring_slot(16), sp_offs + split_blocks(m), 24, hipMemcpyDeviceToHost, E.stream),
                   "hipMemcpyAsync(split count)");
                ck(hipEventRecord(E.sync_event(2), E.stream), "hipEventRecord");
                deferred.active = true;
                deferred.src = U;
                deferred.rows = m;
            };
            // replacement selection: the open run starts at rs_off in the
            // spill buffer and holds rs_rows rows so far
            uint64_t rs_off = 0, rs_rows = 0;
            // memory is full under replacement selection: the merged index
            // idx[target] (m rows) keeps K rows.  The excess rows at or after
            // the cursor (row pc on) end the open run; if the scan passes the
            // largest key, the run ends and the smallest keys start the next.
            // The kept rows go to the front of the other index buffer, the
            // evicted ones behind them, and are copied out on the copy stream.
            auto evict = [&](int target, uint64_t m, uint64_t pc) {
                flush_copy();
                const int o = target ^ 1;
                const uint64_t K = p.capacity, e = m - K;
                const uint64_t a = std::min(e, m - pc), b = e - a;
                const uint64_t bytes = e * sw * 8;
                if (!spill.host_pinned || spill_used + bytes > spill.bytes)
                    throw Fail{ISA_ESPILL, "spill buffer too small"};
                if (pend_buf == o) {
                    ck(hipStreamWaitEvent(E.stream, E.sync_event(1), 0), "hipStreamWaitEvent");
                    pend_buf = -1;
                }
                launch_rs_evict(idx[target], m, (uint32_t)sw, pc, a, b, idx[o], rs_cur, E.stream);
                ck(hipEventRecord(E.sync_event(0), E.stream), "hipEventRecord");
                ck(hipStreamWaitEvent(cs, E.sync_event(0), 0), "hipStreamWaitEvent");
                E.pbegin("spill_d2h", cs);
                ck(hipMemcpyAsync(spill_dev + spill_used, idx[o] + K * sw, bytes, hipMemcpyDeviceToDeviceNoCU, cs),
                   "hipMemcpyAsync(spill)");
                E.pend(e, bytes, cs);
                ck(hipEventRecord(E.sync_event(1), cs), "hipEventRecord");
                pend_buf = o;
                pend_lo = K * sw * 8;
                if (!rs_rows) rs_off = spill_used;
                rs_rows += a;
                if (b) {
                    if (rs_rows) runs.push_back(RunInfo{rs_off, 0, rs_rows});
                    rs_off = spill_used + a * sw * 8;
                    rs_rows = b;
                }
                spill_used += bytes;
                spilled += e;
                spilled_bytes += bytes;
                ip = idx[o];
                n_idx = K;
            };
            // absorb decision for the merge of batch j (g_j rows) into
            // idx[target]: keep the merged index if it holds at most K keys;
            // else spill the old index and start a new one with the batch run
            // (read-sort-write), or evict the excess (replacement selection)
            // Hybrid run generation (Section 5, hybrid algorithms).  The
            // index is one sorted array: the resident rows (keys below the
            // cut) followed by the run-generation rows (keys at or above it).
            // After an absorb, with p resident rows of m: if the run-generation
            // part exceeds Kw, the old index's run-generation part is written
            // as a run and the batch's rows at or above the cut replace it; if
            // the resident part exceeds Kr, its rows beyond the first
            // 3/4 Kr are written as a run (a demotion) and the cut moves down
            // to the first of them.  Runs are compacted into the staging area
            // and copied out on the copy stream.
            uint64_t n_res = 0;  // resident rows of the index
            auto write_runs = [&](const std::vector<std::pair<const uint64_t*, uint64_t>>& rr) {
                if (!spill.host_pinned) throw Fail{ISA_ESPILL, "spill buffer too small"};
                // the staging area's last copy must be done
                ck(hipStreamWaitEvent(E.stream, E.sync_event(1), 0), "hipStreamWaitEvent");
                uint64_t at = 0;
                std::vector<uint64_t> at_of;
                for (size_t r = 0; r < rr.size(); ++r) {
                    at_of.push_back(at);
                    if (compact) {
                        launch_split(rr[r].first, rr[r].second, S, Rl, sp_counts, sp_tiles, sp_offs,
                                     hy_stage + at, 0, E.stream);
                        ck(hipMemcpyAsync(E.ring_slot(16 + r), sp_offs + split_blocks(rr[r].second), 24,
                                          hipMemcpyDeviceToHost, E.stream),
                           "hipMemcpyAsync(split count)");
                    } else {
                        launch_copy_words(rr[r].first, hy_stage + at, rr[r].second * sw, E.stream);
                    }
                    at += rr[r].second * sw;
                }
                ck(hipEventRecord(E.sync_event(2), E.stream), "hipEventRecord");
                ck(hipEventSynchronize(E.sync_event(2)), "hipEventSynchronize(split count)");
                ck(hipStreamWaitEvent(cs, E.sync_event(2), 0), "hipStreamWaitEvent");
                for (size_t r = 0; r < rr.size(); ++r) {
                    const uint64_t n_run = rr[r].second;
                    uint64_t n_single = 0, n_packed = 0, bytes = n_run * sw * 8;
                    bool narrow = false;
                    if (compact) {
                        n_single = ((const uint64_t*)E.ring_slot(16 + r))[0];
                        narrow = ((const uint64_t*)E.ring_slot(16 + r))[1] != 0;
                        n_packed = ((const uint64_t*)E.ring_slot(16 + r))[2];
                        bytes = compact_bytes(n_single, n_packed, n_run - n_single - n_packed, Rl, S, narrow);
                    }
                    if (spill_used + bytes > spill.bytes) throw Fail{ISA_ESPILL, "spill buffer too small"};
                    E.pbegin("spill_d2h", cs);
                    ck(hipMemcpyAsync(spill_dev + spill_used, hy_stage + at_of[r], bytes, hipMemcpyDeviceToDeviceNoCU,
                                      cs),
                       "hipMemcpyAsync(spill)");
                    E.pend(n_run, bytes, cs);
                    RunInfo ri;
                    ri.byte_off = spill_used;
                    ri.n_single = n_single;
                    ri.n_packed = n_packed;
                    ri.n_multi = n_run - n_single - n_packed;
                    ri.narrow = narrow;
                    runs.push_back(ri);
                    spill_used += bytes;
                    spilled += n_run;
                    spilled_bytes += bytes;
                }
                ck(hipEventRecord(E.sync_event(1), cs), "hipEventRecord");
            };
            auto decide_hybrid = [&](uint64_t j, uint64_t gj, int target) {
                const uint64_t* h = (const uint64_t*)rb_merge(j);
                if (h[0] >> 32) throw Fail{ISA_EDEVICE, "merge placement wait timed out"};
                const uint64_t m = h[1], pr = h[2], pb = h[3];
                const bool spill_w = m - pr > Kw;
                const bool demote = pr > Kr;
                uint64_t* U = idx[target];
                if (!spill_w && !demote) {
                    ip = U;
                    n_idx = m;
                    n_res = pr;
                    return;
                }
                const uint64_t q = demote ? Kr * 3 / 4 : pr;  // resident rows kept
                std::vector<std::pair<const uint64_t*, uint64_t>> rr;
                if (spill_w && n_idx > n_res) rr.push_back({ip + n_res * sw, n_idx - n_res});
                if (demote) rr.push_back({U + q * sw, pr - q});
                write_runs(rr);
                if (demote) {
                    launch_copy_words(U + q * sw, rs_cur, 1, E.stream);
                    launch_fill(rs_cur + 1, 1, 0, E.stream);
                }
                uint64_t nw;
                if (spill_w) {
                    nw = gj - pb;
                    launch_copy_words(brun[j % 3] + pb * sw, U + q * sw, nw * sw, E.stream);
                } else {
                    // move the run-generation rows down behind the kept
                    // resident rows, in chunks no longer than the distance
                    nw = m - pr;
                    const uint64_t dist = pr - q;
                    for (uint64_t c = 0; c < nw; c += dist) {
                        const uint64_t len = std::min(dist, nw - c);
                        launch_copy_words(U + (pr + c) * sw, U + (q + c) * sw, len * sw, E.stream);
                    }
                }
                // the batch run and the index are read up to here
                ck(hipEventRecord(ev_merge(j), E.stream), "hipEventRecord");
                ip = U;
                n_res = q;
                n_idx = q + nw;
            };
            auto decide = [&](uint64_t j, uint64_t gj, int target, bool rev) {
                if (hy) return decide_hybrid(j, gj, target);
                const uint64_t* h = (const uint64_t*)rb_merge(j);
                if (h[0] >> 32) throw Fail{ISA_EDEVICE, "merge placement wait timed out"};
                const uint64_t m = h[1];
                if (inplace) {
                    // a reverse merge leaves the index at the buffer's tail
                    uint64_t* U = rev ? idx[0] + (buf_rows - m) * sw : idx[0];
                    if (m <= p.capacity) {
                        ip = U;
                        n_idx = m;
                    } else {
                        spill_inplace(U, m);
                        ip = nullptr;
                        n_idx = 0;
                    }
                    return;
                }
                if (m <= p.capacity) {
                    ip = idx[target];
                    n_idx = m;
                } else if (rs) {
                    evict(target, m, h[2]);
                } else {
                    spill_index();
                    ip = brun[j % 3];
                    n_idx = gj;
                }
            };
            // Batches are sorted on two streams of their own (batch b on
            // ss2[b % 2], with the batch program's scratch set b % 2), so that
            // the sorts of batches i and i+1 overlap each other and the absorb
            // of batch i.  A sort waits for the last absorb that reads the
            // batch-run buffer it overwrites (as the batch run, or as the index
            // that a spill left in it); the first sorts wait for everything
            // enqueued on the main stream before them.  An absorb waits for its
            // batch's sort.
            hipStream_t ss2[2] = {E.side(1), E.side(2)};
            int64_t last_reader[3] = {-1, -1, -1};
            bool merged = false;
            auto sort_batch = [&](uint64_t b) {
                hipStream_t ss = ss2[b % 2];
                if (!merged) {
                    ck(hipEventRecord(E.sync_event(24), E.stream), "hipEventRecord");
                    ck(hipStreamWaitEvent(ss, E.sync_event(24), 0), "hipStreamWaitEvent");
                } else if (last_reader[b % 3] >= 0) {
                    ck(hipStreamWaitEvent(ss, ev_merge((uint64_t)last_reader[b % 3]), 0), "hipStreamWaitEvent");
                }
                bp.enqueue(E, b, (uint32_t)(b % 3), rb_sort(b), ss);
                ck(hipEventRecord(ev_sort(b), ss), "hipEventRecord");
            };
            sort_batch(0);
            bool merge_out = false;  // a merge whose absorb is not decided yet
            uint64_t merge_batch = 0, merge_g = 0;
            int merge_tgt = 0;
            bool merge_rev = false;
            uint64_t n_merges = 0;
            for (uint64_t i = 0; i < bp.batches; ++i) {
                const uint32_t slot = (uint32_t)(i % 3);
                if (i + 1 < bp.batches) sort_batch(i + 1);
                ck(hipEventSynchronize(ev_sort(i)), "hipEventSynchronize");
                if (merge_out) ck(hipEventSynchronize(ev_merge(merge_batch)), "hipEventSynchronize");
                uint64_t g = 0;
                if (!bp.result(rb_sort(i), g)) {
                    // a bucket was too large for a leaf: redo the batch with the
                    // general plan in the batch program's scratch, once the sort
                    // streams (the scratch's other users) are idle; later sorts
                    // wait for the main stream
                    for (hipStream_t ss : ss2) ck(hipStreamSynchronize(ss), "hipStreamSynchronize(sort)");
                    A.off = bp.scratch_off;
                    std::vector<Instance> inst(1);
                    inst[0].src = bp.batch_src(i);
                    inst[0].n = bp.batch_n(i);
                    inst[0].dest = 0;
                    g = sort_reduce(E, A, inst, std::vector<Dest>(1, bdest[slot]), k, false, &hint)[0];
                    A.off = top;
                    // the batch's group count where the device reads it (the
                    // hybrid policy's probe of the batch run)
                    ((uint64_t*)rb_sort(i))[1] = g;
                    ck(hipEventRecord(E.sync_event(25), E.stream), "hipEventRecord");
                    for (hipStream_t ss : ss2) ck(hipStreamWaitEvent(ss, E.sync_event(25), 0), "hipStreamWaitEvent");
                }
                ++batches;
                if (merge_out) {
                    decide(merge_batch, merge_g, merge_tgt, merge_rev);
                    merge_out = false;
                }
                if (!ip) {
                    // the first batch run is the index (all resident under
                    // hybrid run generation, unless no resident index)
                    ip = brun[slot];
                    n_idx = g;
                    n_res = hy && Kr ? g : 0;
                    // a run split just before (the batch after a spill) is
                    // copied out now: waiting for the next absorb would leave
                    // the host link idle for a batch
                    flush_copy();
                    continue;
                }
                const int tgt = merge_target();
                // in place: an index at the buffer's head is merged backwards,
                // ending at the buffer's end; one at its tail (or a batch run)
                // forwards, from the buffer's start
                const bool rev = inplace && ip == idx[0];
                if (inplace)
                    guard_idx();
                else
                    guard(tgt, (n_idx + g) * sw * 8);
                ck(hipStreamWaitEvent(E.stream, ev_sort(i), 0), "hipStreamWaitEvent");
                // merges alternate between the two control blocks (a batch
                // that starts an index after a spill makes no merge)
                uint64_t* m_ctl = m_ctl2[n_merges % 2];
                E.pbegin("k_merge");
                // the merge's last partition (and the probe) write the result
                // words straight to the pinned readback slot
                uint64_t* rb_dev = E.ring_dev_of(rb_merge(i));
                launch_merge(ip, n_idx, brun[slot], g, idx[tgt], S, m_splits, m_ctl + 3, (uint32_t*)m_ctl, m_ctl + 1,
                             E.stream, m_ctl2[(n_merges + 1) % 2], (uint32_t)mctl_words, rb_dev, rev ? buf_rows : 0);
                ++n_merges;
                E.pend(n_idx + g, (n_idx + g) * sw * 8);
                if (rs) launch_rs_probe(idx[tgt], m_ctl + 1, (uint32_t)sw, rs_cur, rb_dev + 2, E.stream);
                if (hy) {
                    // resident rows of the merged index and of the batch run
                    launch_rs_probe(idx[tgt], m_ctl + 1, (uint32_t)sw, rs_cur, rb_dev + 2, E.stream);
                    launch_rs_probe(brun[slot], E.ring_dev_of(rb_sort(i)) + 1, (uint32_t)sw, rs_cur, rb_dev + 3,
                                    E.stream);
                }
                ck(hipEventRecord(ev_merge(i), E.stream), "hipEventRecord");
                merged = true;
                last_reader[slot] = (int64_t)i;
                for (int j = 0; j < 3; ++j)
                    if (ip == brun[j]) last_reader[j] = (int64_t)i;
                flush_copy();
                merge_out = true;
                merge_batch = i;
                merge_g = g;
                merge_tgt = tgt;
                merge_rev = rev;
            }
            if (merge_out) {
                ck(hipEventSynchronize(ev_merge(merge_batch)), "hipEventSynchronize");
                decide(merge_batch, merge_g, merge_tgt, merge_rev);
            }
            flush_copy();
            if (rs_rows) runs.push_back(RunInfo{rs_off, 0, rs_rows});
            if (!runs.empty()) ck(hipStreamSynchronize(cs), "hipStreamSynchronize(copy)");
            for (hipStream_t ss : ss2) ck(hipStreamSynchronize(ss), "hipStreamSynchronize(sort)");
            E.sync();
            const double t1 = now_ms();
            if (stats) {
                stats->batches = batches;
                stats->batch_rows = p.batch_rows;
                stats->index_capacity = p.capacity;
                stats->resident_capacity = hy ? Kr : 0;
                stats->run_capacity = hy ? Kw : p.capacity;
                stats->runs = runs.size();
                stats->spilled_rows = spilled;
                stats->spilled_bytes = spilled_bytes;
                stats->t_rungen_ms = t1 - t0;
            }
            if (runs.empty()) {
                E.pbegin("k_copy_rows");
                launch_copy_rows(aos_view(ip, S), n_idx, output_view(*out, aggs, 0), out->capacity, E.stream);
                E.pend(n_idx, 2 * n_idx * sw * 8);
                E.sync();
                n_groups = n_idx;
            } else {
                // keep only the live index, at the front; everything after it
                // is merge space
                if (ip && ip != idx[0]) {
                    // an index at the buffer's tail moves down in pieces no
                    // longer than the distance (at least a batch)
                    if (inplace && ip > idx[0] && ip < idx[0] + buf_rows * sw) {
                        const uint64_t dist = (uint64_t)(ip - idx[0]) / sw;
                        for (uint64_t c = 0; c < n_idx; c += dist) {
                            const uint64_t len = std::min(dist, n_idx - c);
                            launch_copy_words(ip + c * sw, idx[0] + c * sw, len * sw, E.stream);
                        }
                    } else {
                        launch_copy_words(ip, idx[0], n_idx * sw, E.stream);
                    }
                }
                const uint64_t idx_off = (uint64_t)((char*)idx[0] - A.base);
                A.off = idx_off + n_idx * sw * 8;
                // Preliminary merge steps (Section 4, Example 4): the smallest
                // runs are merged first, so that a final merge of at most F
                // runs remains.  The first step takes just enough runs that
                // every later step merges F; each writes one run of state rows
                // to the spill buffer.  Runs are ranked by rows, then by the
                // order in which they were written.
                std::vector<uint64_t> run_seq(runs.size());
                for (size_t j = 0; j < runs.size(); ++j) run_seq[j] = j;
                uint64_t next_seq = runs.size(), merge_steps = 0, merge_rows = 0;
                auto run_rows = [](const RunInfo& r) { return r.n_single + r.n_packed + r.n_multi; };
                auto run_bytes = [&](const RunInfo& r) {
                    return compact_bytes(r.n_single, r.n_packed, r.n_multi, Rl, S, r.narrow);
                };
                // space of the spill buffer given back by merged runs (offset ->
                // bytes), reused first fit; new space comes after spill_used
                std::map<uint64_t, uint64_t> free_ext;
                auto give_back = [&](uint64_t off, uint64_t bytes) {
                    if (!bytes) return;
                    auto it = free_ext.emplace(off, bytes).first;
                    auto nx = std::next(it);
                    if (nx != free_ext.end() && it->first + it->second == nx->first) {
                        it->second += nx->second;
                        free_ext.erase(nx);
                    }
                    if (it != free_ext.begin()) {
                        auto pv = std::prev(it);
                        if (pv->first + pv->second == it->first) {
                            pv->second += it->second;
                            free_ext.erase(it);
                        }
                    }
                };
                auto take_space = [&](uint64_t bytes) -> uint64_t {
                    for (auto it = free_ext.begin(); it != free_ext.end(); ++it) {
                        if (it->second >= bytes) {
                            const uint64_t off = it->first, rest = it->second - bytes;
                            free_ext.erase(it);
                            if (rest) free_ext[off + bytes] = rest;
                            return off;
                        }
                    }
                    if (spill_used + bytes > spill.bytes) throw Fail{ISA_ESPILL, "spill buffer too small"};
                    const uint64_t off = spill_used;
                    spill_used += bytes;
                    return off;
                };
                auto prelim = [&](uint64_t F) {
                    bool first = true;
                    while (runs.size() > F) {
                        const uint64_t nr = runs.size();
                        const uint64_t extra = (nr - F) % (F - 1);
                        const uint64_t take = first && extra ? extra + 1 : F;
                        first = false;
                        std::vector<size_t> order(nr);
                        for (size_t j = 0; j < nr; ++j) order[j] = j;
                        std::sort(order.begin(), order.end(), [&](size_t x, size_t y) {
                            const uint64_t rx = run_rows(runs[x]), ry = run_rows(runs[y]);
                            return rx != ry ? rx < ry : run_seq[x] < run_seq[y];
                        });
                        std::vector<bool> used(nr, false);
                        std::vector<RunInfo> sel;
                        for (uint64_t j = 0; j < take; ++j) {
                            used[order[j]] = true;
                            sel.push_back(runs[order[j]]);
                        }
                        // the merged run has at most the rows of its inputs
                        uint64_t bound = 0;
                        for (const RunInfo& r : sel) bound += run_rows(r) * sw * 8;
                        RunSink sk;
                        sk.host = (char*)spill.host_pinned;
                        sk.off = take_space(bound);
                        sk.cap = bound;
                        uint64_t g = 0;
                        A.off = idx_off + n_idx * sw * 8;
                        wide_merge(E, A, k, aggs, sel, (const char*)spill.host_pinned, idx[0], 0, out, nullptr, g,
                                   &sk);
                        std::vector<RunInfo> keep;
                        std::vector<uint64_t> keep_seq;
                        for (size_t j = 0; j < nr; ++j)
                            if (!used[j]) {
                                keep.push_back(runs[j]);
                                keep_seq.push_back(run_seq[j]);
                            }
                        keep.push_back(RunInfo{sk.off, 0, sk.rows});
                        keep_seq.push_back(next_seq++);
                        runs.swap(keep);
                        run_seq.swap(keep_seq);
                        // the merged inputs' space and the unused end of the bound
                        give_back(sk.off + sk.rows * sw * 8, bound - sk.rows * sw * 8);
                        for (const RunInfo& r : sel) give_back(r.byte_off, run_bytes(r));
                        ++merge_steps;
                        merge_rows += sk.rows;
                    }
                };
                if (E.tune.merge_fanin && runs.size() > E.tune.merge_fanin) prelim(E.tune.merge_fanin);
                bool halved = false;
                for (;;) {
                    try {
                        A.off = idx_off + n_idx * sw * 8;
                        wide_merge(E, A, k, aggs, runs, (const char*)spill.host_pinned, idx[0], n_idx, out, stats,
                                   n_groups);
                        break;
                    } catch (const Fail& f) {
                        if (f.status != ISA_ESPILL) throw;
                        if (n_idx) {
                            // No window fits beside the final index (a full index
                            // under replacement selection in a small workspace):
                            // write the index out as one more run, which frees its
                            // room, and merge from host memory alone.  Every
                            // spilled state row still stands for at least one
                            // input row, so the spill buffer of one state row per
                            // input row holds it.
                            const uint64_t bytes = n_idx * sw * 8;
                            if (spill_used + bytes > spill.bytes) throw;
                            ck(hipMemcpyAsync(spill_dev + spill_used, idx[0], bytes, hipMemcpyDeviceToDeviceNoCU,
                                              E.stream),
                               "hipMemcpyAsync(spill index)");
                            E.sync();
                            runs.push_back(RunInfo{spill_used, 0, n_idx});
                            run_seq.push_back(next_seq++);
                            spill_used += bytes;
                            spilled += n_idx;
                            spilled_bytes += bytes;
                            if (stats) {
                                stats->runs = runs.size();
                                stats->spilled_rows = spilled;
                                stats->spilled_bytes = spilled_bytes;
                                stats->windows = 0;
                            }
                            n_idx = 0;
                            continue;
                        }
                        // still no window fits all runs: merge the smallest runs
                        // first, down to half as many
                        if (!halved && runs.size() > 2) {
                            halved = true;
                            prelim(std::max<uint64_t>(2, runs.size() / 2));
                            continue;
                        }
                        throw;
                    }
                }
                if (stats) {
                    stats->merge_steps = merge_steps;
                    stats->merge_rows = merge_rows;
                }
            }
            if (stats) {
                stats->peak_ws_bytes = A.peak;
                stats->t_merge_ms = now_ms() - t1;
            }
        }
        out->n_groups = n_groups;
        return n_groups > out->capacity ? ISA_ETRUNC : ISA_OK;
    } catch (const Fail& f) {
        out->n_groups = 0;
        return fail(ctx, f);
    } catch (const std::bad_alloc&) {
        out->n_groups = 0;
        return ISA_ENOMEM;
    }
}

}  // extern "C"

extern "C" {

}  // extern "C"

namespace {

// In-stream grouping of rows already sorted on key >> shift into `ov`
// (capacity cap); returns the number of groups (> cap: nothing written).
// Rows are in raw layout: count 1 or a count column, and one value column for
// sum, min and max.
uint64_t sorted_group(Engine& E, Arena& A, const ColView& V, uint64_t n, int shift, const OutView& ov, uint64_t cap) {
    if (V.mn != V.sum || V.mx != V.sum) throw Fail{ISA_EINVAL, "internal: sorted grouping takes raw rows"};
    const uint64_t m = sorted_tiles(n);
    uint32_t* heads = A.take_n<uint32_t>(m + 1);
    uint64_t* offs = A.take_n<uint64_t>(m + 1);
    uint64_t* tiles = A.take_n<uint64_t>(scan_tiles(m) + 1);
    uint64_t* bounds = A.take_n<uint64_t>(m + 1);
    uint64_t* bigs = A.take_n<uint64_t>(3 * m + 3);
    uint64_t* ctl = A.take_n<uint64_t>(1);  // [bad, n_bigs] as two u32
    launch_fill(ctl, 1, 0, E.stream);
    E.pbegin("k_sorted_tiles");
    launch_sorted_tiles(V, n, shift, heads, (uint32_t*)ctl, E.stream);
    E.pend(n, n * 8);
    launch_scan(heads, m, tiles, offs, E.stream);
    const uint64_t* h = (const uint64_t*)download_async(E, ctl, 8);
    const uint64_t* hg = (const uint64_t*)download_async(E, offs + m, 8);
    E.sync();
    if ((uint32_t)h[0]) throw Fail{ISA_EINVAL, "input is not sorted on the key"};
    const uint64_t groups = *hg;
    if (groups > cap) return groups;
    launch_sorted_align(V, n, shift, bounds, E.stream);
    const uint64_t row_bytes = 8 + (V.cnt ? 8 : 0) + (V.sum ? 8 : 0) + (V.fs ? 8 : 0);
    E.pbegin("k_sorted_ranges");
    launch_sorted_ranges(V, n, shift, bounds, offs, ov, cap, bigs, (uint32_t*)ctl + 1, E.stream);
    E.pend(n, n * row_bytes);
    const uint64_t* hb = (const uint64_t*)download_async(E, ctl, 8);
    E.sync();
    const uint32_t n_bigs = (uint32_t)(hb[0] >> 32);
    if (n_bigs) {
        std::vector<uint64_t> hbig(3 * (size_t)n_bigs);
        const uint64_t* p = (const uint64_t*)download_async(E, bigs, hbig.size() * 8);
        E.sync();
        std::memcpy(hbig.data(), p, hbig.size() * 8);
        Leaf lf;
        std::memset(&lf, 0, sizeof(lf));
        lf.src = V;
        std::vector<SinglePiece> pieces;
        std::vector<uint32_t> first(n_bigs + 1, 0);
        for (uint32_t b = 0; b < n_bigs; ++b) {
            first[b] = (uint32_t)pieces.size();
            for (uint64_t r = hbig[3 * b]; r < hbig[3 * b + 1]; r += SINGLE_CHUNK) {
                SinglePiece sp;
                sp.leaf = 0;
                sp.slot = (uint32_t)pieces.size();
                sp.start = r;
                sp.n = (uint32_t)std::min<uint64_t>(SINGLE_CHUNK, hbig[3 * b + 1] - r);
                sp.pad = 0;
                pieces.push_back(sp);
            }
        }
        first[n_bigs] = (uint32_t)pieces.size();
        UpPack up;
        const uint64_t o_l = up.add(&lf, sizeof(lf));
        const uint64_t o_p = up.add(pieces.data(), pieces.size() * sizeof(SinglePiece));
        const uint64_t o_f = up.add(first.data(), first.size() * sizeof(uint32_t));
        char* d = up.commit(E, A);
        void* partials = A.take(pieces.size() * single_partial_bytes());
        uint64_t big_rows = 0;
        for (uint32_t b = 0; b < n_bigs; ++b) big_rows += hbig[3 * b + 1] - hbig[3 * b];
        E.pbegin("k_single_partial");
        launch_single_partial((const Leaf*)(d + o_l), (const SinglePiece*)(d + o_p), (uint32_t)pieces.size(), partials,
                              E.stream);
        E.pend(big_rows, 0);
        launch_sorted_big_final(V, shift, bigs, n_bigs, (const uint32_t*)(d + o_f), partials, ov, cap, E.stream);
        E.sync();
    }
    return groups;
}

}  // namespace

extern "C" {

uint64_t isa_columns_workspace_bytes(uint64_t n_rows, uint32_t n_cols) {
    if (n_cols == 0 || n_cols > ISA_MAX_KEY_COLUMNS) return 0;
    const uint64_t nb = rdx_blocks(n_rows) + 1;
    const uint64_t hist = nb * 256;
    // two (key, row) buffers, the histogram and its scan, heads and their
    // scan, group numbers, group heads, the value column in sorted order, the
    // sorted grouping's bookkeeping and the column pointer tables
    return n_rows * (2 * 8 + 2 * 4) + hist * 4 + (hist + 1) * 8 + (scan_tiles(hist) + 1) * 8 + n_rows * 4 +
           (n_rows + 1) * 8 + (scan_tiles(n_rows) + 1) * 8 + 3 * n_rows * 8 + (n_rows / 3584 + 8) * 64 +
           (1u << 20);
}

isa_status isa_group_by_columns(isa_ctx* ctx, const int64_t* const* key_cols, uint32_t n_cols,
                                const int64_t* v_i64, uint64_t n_rows, uint32_t aggs, isa_workspace ws,
                                int64_t* const* out_cols, isa_output* out, uint32_t* code_offset,
                                int64_t* code_value, uint64_t* column_compares, void* stream) {
    if (out) out->n_groups = 0;
    if (column_compares) *column_compares = 0;
    if (!ctx || !key_cols || !out_cols || !out || n_cols == 0 || n_cols > ISA_MAX_KEY_COLUMNS) return ISA_EINVAL;
    if ((aggs & ~(uint32_t)(ISA_COUNT | ISA_SUM_I64 | ISA_MIN_I64 | ISA_MAX_I64)) != 0) return ISA_EINVAL;
    if ((aggs & (ISA_SUM_I64 | ISA_MIN_I64 | ISA_MAX_I64)) && !v_i64) return ISA_EINVAL;
    isa_status s = check_output(out, aggs, false);
    if (s != ISA_OK) return s;
    if (n_rows == 0) return ISA_OK;
    if (n_rows > 0xFFFFFFFFull) return ISA_EINVAL;  // rows are numbered in 32 bits
    for (uint32_t c = 0; c < n_cols; ++c)
        if (!key_cols[c] || !out_cols[c]) return ISA_EINVAL;
    if (!ws.dev || ((uintptr_t)ws.dev & 255)) return ISA_EINVAL;
    if (ws.bytes < isa_columns_workspace_bytes(n_rows, n_cols)) return ISA_EBUDGET;
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        ck(hipSetDevice(ctx->device), "hipSetDevice");
        Engine& E = ctx->eng;
        E.stream = (hipStream_t)stream;
        Arena A;
        A.base = (char*)ws.dev;
        A.cap = ws.bytes;
        const uint64_t n = n_rows;
        const uint64_t nb = rdx_blocks(n);
        const uint64_t hn = nb * 256;
        uint64_t* keys[2] = {A.take_n<uint64_t>(n), A.take_n<uint64_t>(n)};
        uint32_t* perm[2] = {A.take_n<uint32_t>(n), A.take_n<uint32_t>(n)};
        uint32_t* hist = A.take_n<uint32_t>(hn);
        uint64_t* hoffs = A.take_n<uint64_t>(hn + 1);
        uint64_t* htiles = A.take_n<uint64_t>(scan_tiles(hn) + 1);
        uint64_t* mm = A.take_n<uint64_t>(2);
        // column pointer tables on the device
        UpPack up;
        const uint64_t o_in = up.add(key_cols, n_cols * sizeof(int64_t*));
        const uint64_t o_out = up.add(out_cols, n_cols * sizeof(int64_t*));
        char* d_up = up.commit(E, A);
        const int64_t* const* d_cols = (const int64_t* const*)(d_up + o_in);
        int64_t* const* d_out_cols = (int64_t* const*)(d_up + o_out);
        // Stable LSD sort of the row order, the last column first; each
        // column's passes cover only the bits in which its values differ.
        const uint32_t* cur_perm = nullptr;  // the identity until a pass moves rows
        int cur = 0;
        for (int c = (int)n_cols - 1; c >= 0; --c) {
            const uint64_t init[2] = {~0ull, 0ull};
            E.upload(mm, init, 16);
            launch_col_minmax(key_cols[c], n, mm, E.stream);
            const uint64_t* h = (const uint64_t*)download_async(E, mm, 16);
            E.sync();
            const uint64_t lo = h[0], range = h[1] - h[0];
            if (range == 0) continue;  // one value: the column orders nothing
            int nbits = 0;
            while (nbits < 64 && (range >> nbits)) ++nbits;
            launch_col_keys(key_cols[c], cur_perm, n, lo, keys[cur], E.stream);
            for (int shift = 0; shift < nbits; shift += 8) {
                E.pbegin("k_rdx_hist");
                launch_rdx_hist(keys[cur], n, shift, hist, E.stream);
                E.pend(n, n * 8);
                launch_scan(hist, hn, htiles, hoffs, E.stream);
                E.pbegin("k_rdx_scatter");
                launch_rdx_scatter(keys[cur], cur_perm, n, shift, hoffs, keys[cur ^ 1], perm[cur ^ 1], E.stream);
                E.pend(n, n * 24);
                cur ^= 1;
                cur_perm = perm[cur];
            }
        }
        // codes against the predecessor decide the group boundaries
        uint32_t* heads = A.take_n<uint32_t>(n);
        uint64_t* goffs = A.take_n<uint64_t>(n + 1);
        uint64_t* gtiles = A.take_n<uint64_t>(scan_tiles(n) + 1);
        uint64_t* cmp = A.take_n<uint64_t>(1);
        launch_fill(cmp, 1, 0, E.stream);
        E.pbegin("k_ovc");
        launch_ovc(d_cols, n_cols, cur_perm, n, heads, code_offset, code_value, cmp, E.stream);
        E.pend(n, n * 8 * n_cols);
        launch_scan(heads, n, gtiles, goffs, E.stream);
        uint64_t* gid = A.take_n<uint64_t>(n);
        uint64_t* head_pos = A.take_n<uint64_t>(n);
        int64_t* vs = v_i64 && (aggs & (ISA_SUM_I64 | ISA_MIN_I64 | ISA_MAX_I64)) ? A.take_n<int64_t>(n) : nullptr;
        launch_group_ids(heads, goffs, cur_perm, vs ? v_i64 : nullptr, n, gid, head_pos, vs, E.stream);
        const uint64_t* hg = (const uint64_t*)download_async(E, goffs + n, 8);
        const uint64_t* hc = (const uint64_t*)download_async(E, cmp, 8);
        E.sync();
        const uint64_t groups = *hg;
        if (column_compares) *column_compares = *hc;
        out->n_groups = groups;
        if (groups > out->capacity) return ISA_ETRUNC;
        launch_group_keys(d_cols, n_cols, cur_perm, head_pos, groups, d_out_cols, E.stream);
        // the aggregates: in-stream grouping of the sorted rows on their group
        // numbers (the sorted-input path)
        const Cols k = cols_of(aggs);
        ColView V;
        V.key = gid;
        V.cnt = nullptr;
        V.sum = V.mn = V.mx = vs;
        V.fs = nullptr;
        V.stride = 1;
        // the sorted path writes a key column: the group numbers go to the
        // first key buffer, free once the rows are ordered
        OutView ov = output_view(*out, aggs, 0);
        ov.key = keys[0];
        (void)k;
        if (aggs) {
            const uint64_t g2 = sorted_group(E, A, V, n, 0, ov, out->capacity);
            if (g2 != groups) throw Fail{ISA_EDEVICE, "internal: group count mismatch"};
        }
        E.sync();
        return ISA_OK;
    } catch (const Fail& f) {
        out->n_groups = 0;
        return fail(ctx, f);
    } catch (const std::bad_alloc&) {
        out->n_groups = 0;
        return ISA_ENOMEM;
    }
}

isa_status isa_group_by_sorted(isa_ctx* ctx, const isa_input* in, uint32_t aggs, isa_workspace ws, isa_output* out,
                               void* stream) {
    if (out) out->n_groups = 0;
    if (!ctx || !valid_aggs(aggs)) return ISA_EINVAL;
    isa_status s = check_input(in, aggs);
    if (s != ISA_OK) return s;
    s = check_output(out, aggs, true);
    if (s != ISA_OK) return s;
    if (in->n_rows == 0) return ISA_OK;
    if (!ws.dev || ((uintptr_t)ws.dev & 255)) return ISA_EINVAL;
    const Cols k = cols_of(aggs);
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        ck(hipSetDevice(ctx->device), "hipSetDevice");
        Engine& E = ctx->eng;
        E.stream = (hipStream_t)stream;
        Arena A;
        A.base = (char*)ws.dev;
        A.cap = ws.bytes;
        const uint64_t g = sorted_group(E, A, input_view(*in, k), in->n_rows, 0, output_view(*out, aggs, 0),
                                        out->capacity);
        out->n_groups = g;
        return g > out->capacity ? ISA_ETRUNC : ISA_OK;
    } catch (const Fail& f) {
        out->n_groups = 0;
        return fail(ctx, f);
    } catch (const std::bad_alloc&) {
        out->n_groups = 0;
        return ISA_ENOMEM;
    }
}

isa_status isa_count_distinct(isa_ctx* ctx, const int32_t* g, const int32_t* x, uint64_t n, isa_workspace ws,
                              isa_spill spill, void* pair_scratch, uint64_t scratch_bytes, int32_t* out_g,
                              uint64_t* out_count, uint64_t* out_distinct, uint64_t capacity, uint64_t* n_groups,
                              void* stream) {
    if (n_groups) *n_groups = 0;
    if (!ctx || !n_groups) return ISA_EINVAL;
    if (n == 0) return ISA_OK;
    if (!g || !x || !out_g || !out_count || !out_distinct || !pair_scratch || ((uintptr_t)pair_scratch & 7))
        return ISA_EINVAL;
    if (scratch_bytes < 8 * n) return ISA_EBUDGET;
    uint64_t* keys = (uint64_t*)pair_scratch;
    const uint64_t pcap = (scratch_bytes - 8 * n) / 16;
    uint64_t* pk = keys + n;
    uint64_t* pc = pk + pcap;
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        try {
            ck(hipSetDevice(ctx->device), "hipSetDevice");
            Engine& E = ctx->eng;
            E.stream = (hipStream_t)stream;
            launch_pack_pairs(g, x, n, keys, E.stream);
            ck(hipGetLastError(), "pack");
        } catch (const Fail& f) {
            return fail(ctx, f);
        }
    }
    // the pairs, grouped with count(*) (the stream orders the packing first)
    isa_input in;
    in.keys = keys;
    in.v_i64 = nullptr;
    in.v_f64 = nullptr;
    in.n_rows = n;
    isa_output po;
    std::memset(&po, 0, sizeof(po));
    po.keys = pk;
    po.count = pc;
    po.capacity = pcap;
    isa_status st = isa_group_by(ctx, &in, ISA_COUNT, ws, spill, &po, nullptr, stream);
    if (st == ISA_ETRUNC) {
        ctx->last_error = "pair scratch below 16 bytes per distinct pair";
        return ISA_EBUDGET;
    }
    if (st != ISA_OK) return st;
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        Engine& E = ctx->eng;
        E.stream = (hipStream_t)stream;
        Arena A;
        A.base = (char*)ws.dev;
        A.cap = ws.bytes;
        ColView V;
        V.key = pk;
        V.cnt = nullptr;
        V.sum = V.mn = V.mx = (const int64_t*)pc;
        V.fs = nullptr;
        V.stride = 1;
        OutView ov;
        ov.key = keys;  // the normalized g, converted below
        ov.cnt = out_distinct;
        ov.sum = (int64_t*)out_count;
        ov.mn = ov.mx = nullptr;
        ov.fs = nullptr;
        ov.stride = 1;
        const uint64_t groups = sorted_group(E, A, V, po.n_groups, 32, ov, capacity);
        *n_groups = groups;
        if (groups > capacity) return ISA_ETRUNC;
        launch_unpack_hi(keys, groups, out_g, E.stream);
        E.sync();
        return ISA_OK;
    } catch (const Fail& f) {
        *n_groups = 0;
        return fail(ctx, f);
    } catch (const std::bad_alloc&) {
        *n_groups = 0;
        return ISA_ENOMEM;
    }
}

isa_status isa_group_by_segmented(isa_ctx* ctx, const int32_t* a, const int32_t* b, const int64_t* v, uint64_t n,
                                  uint32_t aggs, isa_workspace ws, int32_t* out_a, int32_t* out_b, isa_output* out,
                                  void* stream) {
    if (out) out->n_groups = 0;
    if (!ctx || !valid_aggs(aggs) || (aggs & ISA_SUM_F64)) return ISA_EINVAL;
    isa_status s = check_output(out, aggs, false);
    if (s != ISA_OK) return s;
    if (n == 0) return ISA_OK;
    if (!a || !b || !out_a || !out_b) return ISA_EINVAL;
    const Cols k = cols_of(aggs);
    if (k.v && !v) return ISA_EINVAL;
    if (!ws.dev || ((uintptr_t)ws.dev & 255)) return ISA_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        ck(hipSetDevice(ctx->device), "hipSetDevice");
        Engine& E = ctx->eng;
        E.stream = (hipStream_t)stream;
        Arena A;
        A.base = (char*)ws.dev;
        A.cap = ws.bytes;
        // segment starts: positions where a changes (one scan of a)
        constexpr uint32_t CH = 16384;
        const uint64_t nch = (n + CH - 1) / CH;
        uint32_t* d_cnt = A.take_n<uint32_t>(nch + 1);
        uint64_t* d_offs = A.take_n<uint64_t>(nch + 2);
        uint64_t* d_tiles = A.take_n<uint64_t>(scan_tiles(nch) + 1);
        uint32_t* d_bad = d_cnt + nch;
        ck(hipMemsetAsync(d_bad, 0, 4, E.stream), "hipMemsetAsync");
        launch_seg_count(a, n, CH, d_cnt, d_bad, E.stream);
        launch_scan(d_cnt, nch, d_tiles, d_offs, E.stream);
        const uint64_t* h_ns = (const uint64_t*)download_async(E, d_offs + nch, 8);
        const uint32_t* h_bad = (const uint32_t*)download_async(E, d_bad, 4);
        E.sync();
        const uint64_t n_seg = *h_ns;
        if (*h_bad) throw Fail{ISA_EINVAL, "grouping prefix column is not sorted"};
        uint64_t* d_starts = A.take_n<uint64_t>(n_seg);
        launch_seg_write(a, n, CH, d_offs, d_starts, E.stream);
        const uint64_t* h_st = (const uint64_t*)download_async(E, d_starts, n_seg * 8);
        E.sync();
        std::vector<uint64_t> starts(h_st, h_st + n_seg);
        starts.push_back(n);
        A.off = 0;
        A.peak = 0;
        // segments are independent groupings on b; several run together per wave
        const uint64_t per_row = 16 + (sort_reduce_bytes(1, 0, k, false) - (4u << 20));
        // the segments of one wave: [i0, i1) while they fit the workspace
        auto wave_end = [&](uint64_t i0, uint64_t& rows) {
            uint64_t i1 = i0;
            rows = 0;
            while (i1 < n_seg) {
                const uint64_t r = starts[i1 + 1] - starts[i1];
                const uint64_t need = (rows + r) * per_row + (i1 - i0 + 1) * 4608 + (5u << 20);
                if (need > ws.bytes) break;
                rows += r;
                ++i1;
            }
            if (i1 == i0) throw Fail{ISA_EBUDGET, "one segment does not fit the workspace"};
            return i1;
        };
        auto wave_instances = [&](uint64_t i0, uint64_t i1, const uint64_t* keys) {
            std::vector<Instance> inst;
            const uint64_t r0 = starts[i0];
            for (uint64_t i = i0; i < i1; ++i) {
                Instance in;
                in.src.key = keys + (starts[i] - r0);
                in.src.cnt = nullptr;
                in.src.sum = in.src.mn = in.src.mx = k.v ? v + starts[i] : nullptr;
                in.src.fs = nullptr;
                in.src.stride = 1;
                in.n = starts[i + 1] - starts[i];
                in.dest = 0;
                inst.push_back(in);
            }
            return inst;
        };
        uint64_t max_seg = 0;
        for (uint64_t i = 0; i < n_seg; ++i) max_seg = std::max(max_seg, starts[i + 1] - starts[i]);
        const char* sync_env = std::getenv("ISA_SEGMENTED_SYNC");
        if (max_seg <= FLAT_MAX && !(sync_env && sync_env[0] == '1')) {
            // Waves enqueued back to back, no host round trip between them:
            // a wave's groups start at the output row that the previous
            // wave's last leaf wrote to a device word (two words alternate),
            // its normalized keys go to a buffer of its own (indexed from
            // that row) and are unpacked from there; the flat plans' error
            // words are read once at the end.  A plan that failed (a bucket
            // too large for a leaf) sends the call through the waves below,
            // one at a time.
            uint64_t* d_cur = A.take_n<uint64_t>(2);
            launch_fill(d_cur, 2, 0, E.stream);
            const uint64_t mark = A.off;
            std::vector<const uint64_t*> ctls;
            uint64_t w = 0;
            bool ok = true;
            for (uint64_t i0 = 0; i0 < n_seg && ok; ++w) {
                uint64_t rows = 0;
                const uint64_t i1 = wave_end(i0, rows);
                A.off = mark;
                uint64_t* keys = A.take_n<uint64_t>(rows);
                uint64_t* okeys = A.take_n<uint64_t>(rows);
                launch_pack_pairs(a + starts[i0], b + starts[i0], rows, keys, E.stream);
                Dest d;
                d.out = output_view(*out, aggs, 0);
                d.out.key = okeys;
                d.capacity = out->capacity;
                d.base = d_cur + ((w + 1) % 2);
                d.key_local = 1;
                std::vector<uint64_t> g;
                const uint64_t* hc = nullptr;
                sort_reduce_flat(E, A, wave_instances(i0, i1, keys), std::vector<Dest>(1, d), k, false, nullptr,
                                 false, g, d_cur + (w % 2), &hc);
                if (!hc) {
                    ok = false;
                    break;
                }
                ctls.push_back(hc);
                launch_unpack_pairs_at(okeys, rows, d.base, d_cur + (w % 2), out->capacity, out_a, out_b, E.stream);
                i0 = i1;
            }
            const uint64_t* h_end = (const uint64_t*)download_async(E, d_cur + ((w + 1) % 2), 8);
            E.sync();
            for (const uint64_t* hc : ctls) {
                const uint64_t err = hc[0] >> 32;
                if (err & 1) throw Fail{ISA_EDEVICE, "leaf placement wait timed out"};
                if (err & 2) ok = false;
            }
            if (ok) {
                const uint64_t total = *h_end;
                out->n_groups = total;
                return total > out->capacity ? ISA_ETRUNC : ISA_OK;
            }
        }
        uint64_t cursor = 0;
        uint64_t i0 = 0;
        while (i0 < n_seg) {
            uint64_t i1 = i0, rows = 0;
            while (i1 < n_seg) {
                const uint64_t r = starts[i1 + 1] - starts[i1];
                const uint64_t need = (rows + r) * per_row + (i1 - i0 + 1) * 4608 + (5u << 20);
                if (need > ws.bytes) break;
                rows += r;
                ++i1;
            }
            if (i1 == i0) throw Fail{ISA_EBUDGET, "one segment does not fit the workspace"};
            const uint64_t r0 = starts[i0];
            A.off = 0;
            uint64_t* keys = A.take_n<uint64_t>(rows);
            uint64_t* okeys = A.take_n<uint64_t>(rows);
            launch_pack_pairs(a + r0, b + r0, rows, keys, E.stream);
            std::vector<Instance> inst;
            for (uint64_t i = i0; i < i1; ++i) {
                Instance in;
                in.src.key = keys + (starts[i] - r0);
                in.src.cnt = nullptr;
                in.src.sum = in.src.mn = in.src.mx = k.v ? v + starts[i] : nullptr;
                in.src.fs = nullptr;
                in.src.stride = 1;
                in.n = starts[i + 1] - starts[i];
                in.dest = 0;
                inst.push_back(in);
            }
            const uint64_t cap_left = out->capacity > cursor ? out->capacity - cursor : 0;
            Dest d;
            d.out = output_view(*out, aggs, std::min(cursor, out->capacity));
            d.out.key = okeys;
            d.capacity = std::min(cap_left, rows);
            const uint64_t g = run_instances(E, A, inst, std::vector<Dest>(1, d), k, false, nullptr, false)[0];
            launch_unpack_pairs(okeys, std::min(g, d.capacity), out_a + std::min(cursor, out->capacity),
                                out_b + std::min(cursor, out->capacity), E.stream);
            E.sync();
            cursor += g;
            i0 = i1;
        }
        out->n_groups = cursor;
        return cursor > out->capacity ? ISA_ETRUNC : ISA_OK;
    } catch (const Fail& f) {
        out->n_groups = 0;
        return fail(ctx, f);
    } catch (const std::bad_alloc&) {
        out->n_groups = 0;
        return ISA_ENOMEM;
    }
}

uint64_t isa_batch_workspace_bytes(uint32_t n_inst, const isa_input* inst, uint32_t aggs) {
    if (!inst) return 0;
    uint64_t rows = 0;
    for (uint32_t i = 0; i < n_inst; ++i) rows += inst[i].n_rows;
    return sort_reduce_bytes(rows, n_inst, cols_of(aggs), false);
}

isa_status isa_batch_run(isa_ctx* ctx, uint32_t n_inst, const isa_input* inst, uint32_t aggs, isa_workspace ws,
                         isa_output* outs, void* stream) {
    if (!ctx || !valid_aggs(aggs) || (n_inst && (!inst || !outs))) return ISA_EINVAL;
    for (uint32_t i = 0; i < n_inst; ++i) {
        outs[i].n_groups = 0;
        isa_status s = check_input(&inst[i], aggs);
        if (s != ISA_OK) return s;
        s = check_output(&outs[i], aggs, true);
        if (s != ISA_OK) return s;
    }
    if (!n_inst) return ISA_OK;
    if (!ws.dev || ((uintptr_t)ws.dev & 255)) return ISA_EINVAL;
    const Cols k = cols_of(aggs);
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        ck(hipSetDevice(ctx->device), "hipSetDevice");
        Engine& E = ctx->eng;
        E.stream = (hipStream_t)stream;
        Arena A;
        A.base = (char*)ws.dev;
        A.cap = ws.bytes;
        bool trunc = false;
        // size classes: small instances first (flat plan, one graph launch per
        // wave), then large ones (general plan)
        std::vector<uint32_t> order;
        for (uint32_t i = 0; i < n_inst; ++i)
            if (inst[i].n_rows <= FLAT_MAX) order.push_back(i);
        const size_t n_small = order.size();
        for (uint32_t i = 0; i < n_inst; ++i)
            if (inst[i].n_rows > FLAT_MAX) order.push_back(i);
        size_t i0 = 0;
        while (i0 < order.size()) {
            // a wave: instances of one class whose intermediate data fit together
            const bool small = i0 < n_small;
            const size_t lim = small ? n_small : order.size();
            size_t i1 = i0;
            uint64_t rows = 0;
            while (i1 < lim && i1 - i0 < 65536 &&
                   sort_reduce_bytes(rows + inst[order[i1]].n_rows, i1 - i0 + 1, k, false) <= ws.bytes) {
                rows += inst[order[i1]].n_rows;
                ++i1;
            }
            if (i1 == i0) throw Fail{ISA_EBUDGET, "an instance does not fit the workspace"};
            std::vector<Instance> in;
            std::vector<Dest> ds;
            for (size_t x = i0; x < i1; ++x) {
                const uint32_t i = order[x];
                Instance y;
                y.src = input_view(inst[i], k);
                y.n = inst[i].n_rows;
                y.dest = (uint32_t)(x - i0);
                in.push_back(y);
                Dest d;
                d.out = output_view(outs[i], aggs, 0);
                d.capacity = outs[i].capacity;
                ds.push_back(d);
            }
            A.off = 0;
            const std::vector<uint64_t> g = run_instances(E, A, in, ds, k, false, nullptr, small && E.tune.graph);
            for (size_t x = i0; x < i1; ++x) {
                const uint32_t i = order[x];
                outs[i].n_groups = g[x - i0];
                if (g[x - i0] > outs[i].capacity) trunc = true;
            }
            i0 = i1;
        }
        return trunc ? ISA_ETRUNC : ISA_OK;
    } catch (const Fail& f) {
        return fail(ctx, f);
    } catch (const std::bad_alloc&) {
        return ISA_ENOMEM;
    }
}

namespace {
bool valid_tuning(const isa_tuning& t) {
    // leaves up to half the leaf capacity on average keep sampled buckets within it
    return t.leaf_rows >= 256 && t.leaf_rows <= (uint32_t)LEAF_CAP / 2 && t.chunk_split >= 64 &&
           t.chunk_split <= 4096 && t.graph <= 1 && (t.merge_fanin == 0 || (t.merge_fanin >= 2 && t.merge_fanin <= 65536));
}
}  // namespace

isa_status isa_set_resident_share(isa_ctx* ctx, uint32_t permille) {
    if (!ctx || permille > 1000) return ISA_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->resident_permille = permille;
    return ISA_OK;
}

isa_status isa_set_run_generation(isa_ctx* ctx, int policy) {
    if (!ctx || (policy != ISA_RUNGEN_READ_SORT_WRITE && policy != ISA_RUNGEN_REPLACEMENT &&
                 policy != ISA_RUNGEN_HYBRID))
        return ISA_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->rungen = policy;
    return ISA_OK;
}

int isa_get_run_generation(isa_ctx* ctx) {
    if (!ctx) return -1;
    std::lock_guard<std::mutex> lock(ctx->mu);
    return ctx->rungen;
}

isa_status isa_get_tuning(isa_ctx* ctx, isa_tuning* out) {
    if (!ctx || !out) return ISA_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    out->leaf_rows = ctx->eng.tune.leaf_rows;
    out->chunk_split = ctx->eng.tune.chunk_split;
    out->graph = ctx->eng.tune.graph;
    out->merge_fanin = ctx->eng.tune.merge_fanin;
    return ISA_OK;
}

isa_status isa_set_tuning(isa_ctx* ctx, const isa_tuning* t) {
    if (!ctx || !t || !valid_tuning(*t)) return ISA_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->eng.tune.leaf_rows = t->leaf_rows;
    ctx->eng.tune.chunk_split = t->chunk_split;
    ctx->eng.tune.graph = t->graph;
    ctx->eng.tune.merge_fanin = t->merge_fanin;
    return ISA_OK;
}

uint32_t isa_tune_candidates(isa_tuning* out, uint32_t max) {
    static const uint32_t leaf[] = {1024, 1536, 2048};
    static const uint32_t split[] = {256, 512, 1024};
    uint32_t c = 0;
    for (uint32_t g = 0; g < 2; ++g)
        for (uint32_t l : leaf)
            for (uint32_t sp : split) {
                if (out && c < max) out[c] = isa_tuning{l, sp, 1 - g, 0};
                ++c;
            }
    return c;
}

isa_status isa_tune_batch(isa_ctx* ctx, uint32_t n_inst, const isa_input* inst, uint32_t aggs, isa_workspace ws,
                          isa_output* outs, void* stream, isa_tuning* best, double* times_ms, uint32_t n_times) {
    if (!ctx) return ISA_EINVAL;
    isa_tuning prev;
    isa_get_tuning(ctx, &prev);
    const uint32_t nc = isa_tune_candidates(nullptr, 0);
    std::vector<isa_tuning> cand(nc);
    isa_tune_candidates(cand.data(), nc);
    double best_ms = 0;
    uint32_t best_i = 0;
    for (uint32_t c = 0; c < nc; ++c) {
        isa_set_tuning(ctx, &cand[c]);
        double ms = 0;
        for (int rep = 0; rep < 2; ++rep) {
            const double t0 = now_ms();
            const isa_status st = isa_batch_run(ctx, n_inst, inst, aggs, ws, outs, stream);
            const double t = now_ms() - t0;
            if (st != ISA_OK) {
                isa_set_tuning(ctx, &prev);
                return st;
            }
            ms = rep == 0 ? t : std::min(ms, t);
        }
        if (times_ms && c < n_times) times_ms[c] = ms;
        if (c == 0 || ms < best_ms) {
            best_ms = ms;
            best_i = c;
        }
    }
    isa_set_tuning(ctx, &cand[best_i]);
    if (best) *best = cand[best_i];
    return ISA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: continuous batching of group-by requests against a workspace cap.
// ---------------------------------------------------------------------------

#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

namespace {

struct Req {
    uint64_t ticket;
    isa_input in;
    uint32_t aggs;
    isa_output* out;
    uint64_t need;  // workspace bytes when run alone
    double t_submit = 0, t_done = 0;
    isa_status status = ISA_OK;
    bool done = false;
};

// First-fit allocator over [0, cap) of the server's workspace.
struct Ledger {
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    uint64_t used = 0;
    void init(uint64_t cap) { free_[0] = cap; }
    bool alloc(uint64_t bytes, uint64_t& off) {
        bytes = (bytes + 255) & ~(uint64_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const uint64_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + 255) & ~(uint64_t)255;
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

constexpr uint32_t SERVER_MAX_BATCH = 1024;

}  // namespace

struct isa_server {
    isa_ctx* ctx = nullptr;
    char* ws = nullptr;
    uint64_t cap = 0;
    std::mutex mu;
    std::condition_variable cv;       // work or memory became available
    std::condition_variable cv_done;  // a request finished
    std::deque<Req*> queue;
    std::unordered_map<uint64_t, Req*> reqs;
    uint64_t next_ticket = 1;
    uint32_t running = 0;
    bool stop = false;
    Ledger ledger;
    std::vector<std::thread> workers;
    std::vector<Engine*> engines;
};

namespace {

// Take the longest FIFO prefix of the queue with one aggregate set whose
// combined workspace can be reserved now.
bool take_batch(isa_server* S, std::vector<Req*>& batch, uint64_t& off, uint64_t& bytes) {
    if (S->queue.empty()) return false;
    const uint32_t aggs = S->queue.front()->aggs;
    const Cols k = cols_of(aggs);
    uint64_t rows = 0;
    size_t cnt = 0;
    while (cnt < S->queue.size() && cnt < SERVER_MAX_BATCH && S->queue[cnt]->aggs == aggs &&
           sort_reduce_bytes(rows + S->queue[cnt]->in.n_rows, cnt + 1, k, false) <= S->cap) {
        rows += S->queue[cnt]->in.n_rows;
        ++cnt;
    }
    while (cnt > 0) {
        bytes = sort_reduce_bytes(rows, cnt, k, false);
        if (S->ledger.alloc(bytes, off)) break;
        --cnt;
        rows -= S->queue[cnt]->in.n_rows;
    }
    if (cnt == 0) return false;
    batch.assign(S->queue.begin(), S->queue.begin() + cnt);
    S->queue.erase(S->queue.begin(), S->queue.begin() + cnt);
    return true;
}

void worker_loop(isa_server* S, Engine* E) {
    hipSetDevice(S->ctx->device);
    for (;;) {
        std::vector<Req*> batch;
        uint64_t off = 0, bytes = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || take_batch(S, batch, off, bytes); });
            if (batch.empty()) return;  // stop requested and nothing admitted
            S->running++;
        }
        isa_status st = ISA_OK;
        std::vector<uint64_t> g(batch.size(), 0);
        try {
            const Cols k = cols_of(batch[0]->aggs);
            std::vector<Instance> in;
            std::vector<Dest> ds;
            for (size_t i = 0; i < batch.size(); ++i) {
                Instance x;
                x.src = input_view(batch[i]->in, k);
                x.n = batch[i]->in.n_rows;
                x.dest = (uint32_t)i;
                in.push_back(x);
                Dest d;
                d.out = output_view(*batch[i]->out, batch[i]->aggs, 0);
                d.capacity = batch[i]->out->capacity;
                ds.push_back(d);
            }
            Arena A;
            A.base = S->ws + off;
            A.cap = bytes;
            g = run_instances(*E, A, in, ds, k, false, nullptr, false);
        } catch (const Fail& f) {
            st = (isa_status)f.status;
        } catch (const std::bad_alloc&) {
            st = ISA_ENOMEM;
        }
        const double t = now_ms();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (size_t i = 0; i < batch.size(); ++i) {
                Req* r = batch[i];
                r->out->n_groups = st == ISA_OK ? g[i] : 0;
                r->status = st != ISA_OK ? st : (g[i] > r->out->capacity ? ISA_ETRUNC : ISA_OK);
                r->t_done = t;
                r->done = true;
            }
            S->ledger.release(off, bytes);
            S->running--;
        }
        S->cv.notify_all();
        S->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

isa_status isa_server_create(isa_ctx* ctx, void* workspace, uint64_t hbm_cap_bytes, uint32_t slots,
                             isa_server** out) {
    if (!out) return ISA_EINVAL;
    *out = nullptr;
    if (!ctx || !workspace || ((uintptr_t)workspace & 255) || slots == 0 || slots > 16) return ISA_EINVAL;
    if (hbm_cap_bytes < (16u << 20)) return ISA_EBUDGET;
    isa_server* S = new (std::nothrow) isa_server();
    if (!S) return ISA_ENOMEM;
    S->ctx = ctx;
    S->ws = (char*)workspace;
    S->cap = hbm_cap_bytes;
    S->ledger.init(hbm_cap_bytes);
    if (hipSetDevice(ctx->device) != hipSuccess) {
        delete S;
        return ISA_EDEVICE;
    }
    for (uint32_t i = 0; i < slots; ++i) {
        Engine* E = new Engine();
        E->device = ctx->device;
        if (hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking) != hipSuccess) {
            delete E;
            isa_server_destroy(S);
            return ISA_EDEVICE;
        }
        S->engines.push_back(E);
    }
    for (Engine* E : S->engines) S->workers.emplace_back(worker_loop, S, E);
    *out = S;
    return ISA_OK;
}

isa_status isa_server_submit(isa_server* S, const isa_input* in, uint32_t aggs, isa_output* out, uint64_t* ticket) {
    if (!S || !ticket || !valid_aggs(aggs)) return ISA_EINVAL;
    isa_status s = check_input(in, aggs);
    if (s != ISA_OK) return s;
    s = check_output(out, aggs, true);
    if (s != ISA_OK) return s;
    Req* r = new (std::nothrow) Req();
    if (!r) return ISA_ENOMEM;
    r->in = *in;
    r->aggs = aggs;
    r->out = out;
    r->need = sort_reduce_bytes(in->n_rows, 1, cols_of(aggs), false);
    if (r->need > S->cap) {
        delete r;
        return ISA_ENOMEM;
    }
    out->n_groups = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next_ticket++;
        r->t_submit = now_ms();
        S->reqs[r->ticket] = r;
        S->queue.push_back(r);
        *ticket = r->ticket;
    }
    S->cv.notify_all();
    return ISA_OK;
}

isa_status isa_server_poll(isa_server* S, uint64_t ticket, int* done, double* latency_ms) {
    if (!S || !done) return ISA_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return ISA_EINVAL;
    Req* r = it->second;
    *done = r->done ? 1 : 0;
    if (!r->done) return ISA_OK;
    if (latency_ms) *latency_ms = r->t_done - r->t_submit;
    return r->status;
}

isa_status isa_server_release(isa_server* S, uint64_t ticket) {
    if (!S) return ISA_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return ISA_EINVAL;
    if (!it->second->done) return ISA_EBUSY;
    delete it->second;
    S->reqs.erase(it);
    return ISA_OK;
}

isa_status isa_server_drain(isa_server* S) {
    if (!S) return ISA_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->queue.empty() && S->running == 0; });
    return ISA_OK;
}

void isa_server_destroy(isa_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (std::thread& t : S->workers) t.join();
    for (Engine* E : S->engines) {
        if (E->stream) hipStreamDestroy(E->stream);
        E->release();
        delete E;
    }
    for (auto& kv : S->reqs) delete kv.second;
    delete S;
}

}  // extern "C"
