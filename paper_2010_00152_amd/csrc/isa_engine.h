// Host engine of the grouping library: workspace carving, the multi-level
// partition driver ("sort-reduce"), run generation and the wide merge.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "isa_internal.h"

namespace isa {

// ---- kernel launch wrappers (isa_kernels.hip) ----
void launch_sample(const Region* regions, uint32_t n_regions, uint64_t* splitters, hipStream_t st);
void launch_hist(const Region* regions, const Chunk* chunks, uint32_t n_chunks, const uint64_t* splitters,
                 uint32_t* hist, hipStream_t st);
// hist_self (optional, one region only): the raw histogram; the scatter then
// derives the chunk offsets itself (no scan launch) and writes them to
// offs_out for the launches after it.  max_chunk_rows: the largest chunk's
// rows when known (it picks the tile size), else 0.
void launch_scatter(const Region* regions, const Chunk* chunks, uint32_t n_chunks, const uint64_t* splitters,
                    const uint64_t* offs, uint64_t* dst, Layout L, hipStream_t st,
                    const uint32_t* hist_self = nullptr, uint64_t* offs_out = nullptr, uint64_t max_chunk_rows = 0);
void launch_bucket_starts(const Region* regions, uint32_t n_regions, const uint64_t* offs, const uint64_t* bs_base,
                          uint64_t* bstart, hipStream_t st);
void launch_fill(uint64_t* p, uint64_t n, uint64_t value, hipStream_t st);
uint64_t sorted_tiles(uint64_t n);
void launch_sorted_tiles(ColView V, uint64_t n, int shift, uint32_t* heads, uint32_t* bad, hipStream_t st);
void launch_sorted_align(ColView V, uint64_t n, int shift, uint64_t* bounds, hipStream_t st);
void launch_sorted_ranges(ColView V, uint64_t n, int shift, const uint64_t* bounds, const uint64_t* offs, OutView out,
                          uint64_t cap, uint64_t* bigs, uint32_t* n_bigs, hipStream_t st);
void launch_sorted_big_final(ColView V, int shift, const uint64_t* bigs, uint32_t n_bigs, const uint32_t* first,
                             const void* partials, OutView out, uint64_t cap, hipStream_t st);
void launch_sample_keys(ColView src, uint64_t n, uint64_t S, uint64_t* out, hipStream_t st);
void launch_copy_words(const uint64_t* src, uint64_t* dst, uint64_t n, hipStream_t st);
void launch_extract_keys(const uint64_t* rows, uint64_t n, uint32_t stride, uint64_t* keys, hipStream_t st);
// Histogram of one run-generation batch that also stores its region
// descriptor at reg and clears its control block (ctl_words words).
void launch_hist_batch(const Region& r, Region* reg, uint64_t* ctl, uint32_t ctl_words, const Chunk* chunks,
                       uint32_t n_chunks, const uint64_t* splitters, uint32_t* hist, hipStream_t st);
void launch_leaf(const Leaf* leaves, uint32_t n_leaves, const uint32_t* leaf_dest, const uint32_t* first_seg,
                 const Dest* dests, const void* partials, uint64_t* status, uint64_t* totals, uint32_t* ctl,
                 hipStream_t st);
void launch_leaf_flat(const FlatSlot* slots, uint32_t n_slots, const FlatInst* insts, const Region* regions,
                      const uint64_t* splitters, const uint64_t* offs, const uint64_t* part, Layout L,
                      const uint32_t* first_slot, const Dest* dests, uint64_t* status, uint64_t* totals,
                      uint32_t* ctl, hipStream_t st, const uint32_t* single_of = nullptr,
                      const void* partials = nullptr, uint32_t max_pieces = 0, uint64_t* host_out = nullptr);
void launch_flat_single_partial(const Region* regions, const uint64_t* offs, const uint64_t* part, Layout L,
                                const uint32_t* single_buckets, uint32_t n_single, uint32_t max_pieces, void* partials,
                                hipStream_t st);
void launch_single_partial(const Leaf* leaves, const SinglePiece* pieces, uint32_t n_pieces, void* partials,
                           hipStream_t st);
size_t single_partial_bytes();
uint64_t merge_parts(uint64_t na, uint64_t nb);
// next_ctl (optional): next_words words cleared by the merge for the next one.
// rev_cap > 0: the merged rows end at row rev_cap of out (reverse order of
// partitions); A may then occupy the start of out.  With rev_cap == 0, A may
// occupy the tail of out (in-place absorption; see the kernel).
void launch_merge(const uint64_t* A, uint64_t na, const uint64_t* B, uint64_t nb, uint64_t* out, Layout L,
                  uint64_t* splits, uint64_t* status, uint32_t* ctl, uint64_t* total_out, hipStream_t st,
                  uint64_t* next_ctl = nullptr, uint32_t next_words = 0, uint64_t* host_out = nullptr,
                  uint64_t rev_cap = 0);
// Replacement selection: cursor position in the merged index (*p_out) and
// eviction of rows [p, p+a) and [0, b) (see the kernels).
void launch_rs_probe(const uint64_t* U, const uint64_t* m_ptr, uint32_t w, const uint64_t* cur, uint64_t* p_out,
                     hipStream_t st);
void launch_rs_evict(const uint64_t* U, uint64_t m, uint32_t w, uint64_t p, uint64_t a, uint64_t b, uint64_t* out,
                     uint64_t* cur, hipStream_t st);
uint64_t split_blocks(uint64_t n);
// cap_words > 0: the run is written only if it takes at most that many words.
void launch_split(const uint64_t* rows, uint64_t n, Layout S, Layout R, uint32_t* counts, uint64_t* tiles,
                  uint64_t* offs, uint64_t* out, uint64_t end_words, hipStream_t st, uint64_t cap_words = 0);
void launch_gather(const GatherTask* tasks, uint32_t n_tasks, Layout R, Layout S, uint64_t* dst, hipStream_t st);
void launch_copy_rows(ColView src, uint64_t n, OutView dst, uint64_t cap, hipStream_t st);
uint64_t scan_tiles(uint64_t n);
void launch_scan(const uint32_t* in, uint64_t n, uint64_t* tile_sums, uint64_t* offs, hipStream_t st);
void launch_pack_pairs(const int32_t* a, const int32_t* b, uint64_t n, uint64_t* keys, hipStream_t st);
void launch_unpack_hi(const uint64_t* hi, uint64_t n, int32_t* a, hipStream_t st);
void launch_unpack_pairs(const uint64_t* keys, uint64_t n, int32_t* a, int32_t* b, hipStream_t st);
// Output rows [*lo, *hi) below cap (lo null: 0) from a launch-local key
// buffer of at most max_n keys; the bounds are read on the device.
void launch_unpack_pairs_at(const uint64_t* keys, uint64_t max_n, const uint64_t* lo, const uint64_t* hi,
                            uint64_t cap, int32_t* a, int32_t* b, hipStream_t st);
void launch_seg_count(const int32_t* a, uint64_t n, uint32_t chunk, uint32_t* counts, uint32_t* bad,
                      hipStream_t st);
void launch_seg_write(const int32_t* a, uint64_t n, uint32_t chunk, const uint64_t* offs, uint64_t* starts,
                      hipStream_t st);

// Pinned staging and synchronisation events set up once per context for the
// entry point that must not allocate (enough for every call it accepts).
constexpr uint64_t NOALLOC_PINNED_BYTES = 8ull << 20;
constexpr size_t NOALLOC_EVENTS = 32;

// Device address of the library-owned scratch (NOALLOC_SCRATCH_BYTES) on
// `device`, which must be current; looked up once per device.
hipError_t noalloc_scratch(int device, void** out);

// Multi-column keys: LSD radix sort of a row permutation and offset-value
// codes of the sorted stream (see the kernels).
uint64_t rdx_blocks(uint64_t n);
void launch_col_minmax(const int64_t* col, uint64_t n, uint64_t* out, hipStream_t st);
void launch_col_keys(const int64_t* col, const uint32_t* perm, uint64_t n, uint64_t lo, uint64_t* keys,
                     hipStream_t st);
void launch_rdx_hist(const uint64_t* keys, uint64_t n, int shift, uint32_t* hist, hipStream_t st);
void launch_rdx_scatter(const uint64_t* keys, const uint32_t* perm, uint64_t n, int shift, const uint64_t* offs,
                        uint64_t* keys_out, uint32_t* perm_out, hipStream_t st);
void launch_ovc(const int64_t* const* cols, uint32_t K, const uint32_t* perm, uint64_t n, uint32_t* heads,
                uint32_t* code_off, int64_t* code_val, uint64_t* compares, hipStream_t st);
void launch_group_ids(const uint32_t* heads, const uint64_t* offs, const uint32_t* perm, const int64_t* v,
                      uint64_t n, uint64_t* gid, uint64_t* head_pos, int64_t* v_sorted, hipStream_t st);
void launch_group_keys(const int64_t* const* cols, uint32_t K, const uint32_t* perm, const uint64_t* head_pos,
                       uint64_t groups, int64_t* const* out_cols, hipStream_t st);

// Error carried out of the engine as an isa_status value.
struct Fail {
    int status;
    std::string what;
};

// Which aggregate columns flow through the path.
struct Cols {
    bool c, v, f;  // count, int64 (sum/min/max), float64 sum
};

Layout raw_layout(const Cols& k);
Layout state_layout(const Cols& k);
ColView aos_view(const uint64_t* base, const Layout& L);
OutView aos_out(uint64_t* base, const Layout& L);

// Bump allocator over the caller's workspace.
struct Arena {
    char* base = nullptr;
    uint64_t cap = 0;
    uint64_t off = 0;
    uint64_t peak = 0;
    void* take(uint64_t bytes);  // throws Fail(ISA_EBUDGET) when exhausted
    template <class T>
    T* take_n(uint64_t n) { return (T*)take(n * sizeof(T)); }
    uint64_t left() const { return cap > off ? cap - off : 0; }
};

// Per-kernel launch timing (HIP events on the launch stream), off by default.
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
    uint64_t rows;   // units the launch processed
    uint64_t bytes;  // algorithmic bytes of those units (rows read once)
};

// Per-context host state.
// Launch configuration of the sort-reduce plans (the autotuner's search space).
struct Tuning {
    uint32_t leaf_rows = 2048;  // target rows per leaf bucket (buckets = rows / leaf_rows, 2..MAX_BUCKETS)
    uint32_t chunk_split = 512; // partition chunks per region: chunk rows = rows / chunk_split, in [PART_TILE, PART_CHUNK] (batches of run generation: from PART_CHUNK_MIN)
    uint32_t graph = 1;         // batched waves of small instances launch as one captured graph
    uint32_t merge_fanin = 0;   // runs per merge step of a spilling group-by (0: all in one wide merge)
};

struct Engine {
    int device = 0;
    Tuning tune;
    hipStream_t stream = nullptr;
    // pinned host staging for descriptor uploads and small readbacks
    char* pinned = nullptr;
    uint64_t pinned_cap = 0;
    uint64_t pinned_used = 0;
    std::vector<char*> retired;
    bool prof_on = false;
    // set while an entry point that must not allocate runs: growing a pinned
    // buffer, creating a stream or an event, or capturing a graph then fails
    // with ISA_ENOMEM instead of allocating
    bool no_alloc = false;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;

    // second stream for host-link copies that overlap compute, and events
    hipStream_t copy_stream = nullptr;
    hipStream_t side_streams[3] = {nullptr, nullptr, nullptr};  // extra copy queues
    hipStream_t capture_stream = nullptr;                       // graph capture only
    std::vector<hipEvent_t> sync_events;

    // small pinned ring for readbacks that stay in flight across host waits
    // (slots of 64 bytes, allocated once)
    char* ring = nullptr;
    char* ring_dev_base = nullptr;
    char* ring_slot(size_t i);
    uint64_t* ring_dev(size_t i);  // the slot's device mapping
    uint64_t* ring_dev_of(const char* slot) { return ring_dev((size_t)(slot - ring) / 64); }
    // pinned host table for uploads that stay in flight across syncs of the
    // main stream (the wide merge's gather tasks); grows, never shrinks
    char* table = nullptr;
    uint64_t table_cap = 0;
    void* table_buf(uint64_t bytes);

    void* pinned_buf(uint64_t bytes);
    void upload(void* dev, const void* host, uint64_t bytes);
    void sync();
    // wait for every stream of the engine, ignoring errors (after a failed
    // call, so that no work still reads or writes the caller's buffers)
    void drain();
    void release();
    // allocate, once, what the no-allocation entry point uses: the pinned
    // staging, the readback ring and the synchronisation events
    void prepare_no_alloc();
    hipStream_t copier();             // created on first use
    hipStream_t side(int i);          // extra copy streams 0..2, created on first use
    hipStream_t capturer();           // private stream for graph capture
    hipEvent_t sync_event(size_t i);  // i-th reusable synchronisation event
    // bracket one launch or copy on `st` (default: stream); no-ops unless
    // profiling is on
    void pbegin(const char* name, hipStream_t st = nullptr);
    void pend(uint64_t rows, uint64_t bytes, hipStream_t st = nullptr);
};

// One independent grouping problem of a sort-reduce call.
struct Instance {
    ColView src;
    uint64_t n;
    uint32_t dest;  // index into the dest list
};

// Splitters chosen once for a whole input and reused for each of its batches:
// 255 entries (padded with UINT64_MAX), on the device and on the host.
struct SplitterHint {
    const uint64_t* dev = nullptr;
    const uint64_t* host = nullptr;
    uint32_t nb = 0;
    const double* share = nullptr;  // optional: each bucket's share of the sample
};

// Collects several host arrays into one pinned staging block and uploads them
// with a single copy into one workspace block.
struct UpPack {
    struct Part {
        const void* src;
        uint64_t bytes, off;
    };
    std::vector<Part> parts;
    uint64_t total = 0;
    uint64_t add(const void* src, uint64_t bytes);  // returns the part's offset
    char* commit(Engine& E, Arena& A);              // device base of the block
};

// Choose splitters for `src` (n rows) with nb buckets from a sample of its keys.
// *light_share (optional): the largest sampled share of rows in a bucket that
// spans more than one key.
void choose_splitters(Engine& E, Arena& A, const ColView& src, uint64_t n, uint32_t nb, uint64_t* dev_out,
                      std::vector<uint64_t>& host_out, std::vector<double>* share = nullptr,
                      double* light_share = nullptr);

// Sort and reduce every instance: the sorted unique state rows of instance i
// are appended, in instance order, to dests[instance.dest].  Returns the
// number of groups written (or required) per dest.
std::vector<uint64_t> sort_reduce(Engine& E, Arena& A, const std::vector<Instance>& inst,
                                  const std::vector<Dest>& dests, const Cols& k, bool state_rows,
                                  const SplitterHint* hint = nullptr);
uint32_t buckets_for(const Engine& E, uint64_t n);
uint64_t chunk_rows(const Engine& E, uint64_t n, uint64_t min_rows);

// Device-to-host copy into pinned staging; valid after the next sync().
const void* download_async(Engine& E, const void* dev, uint64_t bytes);

// The flat plan (one partition level, buckets are leaves, no host round trip
// until the end): every instance must have at most FLAT_MAX rows.  With
// `graph` the launch sequence is captured and launched as one HIP graph.
// Returns false, having written nothing reliable, when a bucket turned out too
// large for a leaf; the caller then uses sort_reduce.
// ext_totals (optional): device words that receive each destination's end
// row instead of the plan's own control block.  async_ctl (optional): the
// call returns once the launches are enqueued, leaving totals empty;
// *async_ctl then points at the plan's pinned control-word readback (error
// word first), valid after the stream is synchronised and until the next
// Engine::sync.  Synchronous calls return false when a bucket is too large.
bool sort_reduce_flat(Engine& E, Arena& A, const std::vector<Instance>& inst, const std::vector<Dest>& dests,
                      const Cols& k, bool state_rows, const SplitterHint* hint, bool graph,
                      std::vector<uint64_t>& totals, uint64_t* ext_totals = nullptr,
                      const uint64_t** async_ctl = nullptr);

// The batches of one input sorted and reduced with the flat plan and fixed
// splitters, every launch parameter prepared up front: batch i covers input
// rows [i*Bt, min(n, (i+1)*Bt)) and its sorted unique state rows go to
// dest[slot].  enqueue() launches one batch without any host round trip and
// queues the readback of its control words into a ring slot; result() reads
// them once that copy has completed.
struct BatchProgram {
    uint64_t n = 0, Bt = 0, batches = 0;
    uint32_t nb = 0, chunks_full = 0, chunks_last = 0;
    uint64_t crow = 0;  // rows per partition chunk
    Layout L{};
    ColView src{};
    const uint64_t* splitters = nullptr;
    Region* d_regs = nullptr;  // region ring (one per batch in flight)
    Chunk* d_chunks_full = nullptr;
    Chunk* d_chunks_last = nullptr;
    FlatSlot* d_slots = nullptr;
    uint32_t* d_first = nullptr;
    Dest* d_dests = nullptr;
    uint64_t* d_ctl = nullptr;  // ring of per-batch [ticket|error, total, status x nb]
    uint64_t scratch_off = 0;   // arena offset of the per-batch scratch (reusable by a fallback)
    // Two batches are sorted at once (on two streams), batch i with scratch
    // set i % SETS: a sort's kernels wait on memory with one workgroup per
    // compute unit, and a second batch fills the gaps.
    static constexpr int SETS = 2;
    uint64_t* part[SETS] = {};
    uint32_t* d_hist[SETS] = {};
    uint64_t* d_offs[SETS] = {};
    // single-key buckets (known from the splitters): their pieces are reduced
    // in parallel before the leaves combine them
    uint32_t n_single = 0, max_pieces = 0;
    uint32_t* d_single_list = nullptr;  // bucket of each single-key bucket
    uint32_t* d_single_of = nullptr;    // per bucket: its index in the list, or ~0
    void* d_partials[SETS] = {};
    uint64_t ctl_words() const { return 2 + (uint64_t)nb; }
    void setup(Engine& E, Arena& A, const ColView& src, uint64_t n_rows, uint64_t batch_rows, const Cols& k,
               const SplitterHint& hint, const std::vector<Dest>& dests);
    void enqueue(Engine& E, uint64_t i, uint32_t slot, char* readback, hipStream_t st);
    // false when a bucket was too large for a leaf (the batch must be redone)
    bool result(const char* readback, uint64_t& groups) const;
    uint64_t batch_n(uint64_t i) const { return i + 1 < batches ? Bt : n - i * Bt; }
    ColView batch_src(uint64_t i) const;
};
// Workspace of a BatchProgram, including room for the general plan of one batch.
uint64_t batch_program_bytes(uint64_t Bt, const Cols& k);

// Workspace bytes sort_reduce_flat needs for `rows` rows in n_inst instances.
uint64_t flat_bytes(uint64_t rows, uint64_t n_inst, const Cols& k, bool state_rows);

// Workspace bytes sort_reduce needs for `rows` input rows.
uint64_t sort_reduce_bytes(uint64_t rows, uint64_t n_inst, const Cols& k, bool state_rows);

}  // namespace isa
