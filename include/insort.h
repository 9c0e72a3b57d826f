/*
 * insort.h -- C ABI of a GPU (AMD MI355X, gfx950) implementation of
 * sort-based duplicate removal, grouping and aggregation for unsorted input
 * with early aggregation during run generation and wide merging
 * (Do, Graefe, Naughton, "Efficient sorting, duplicate removal, grouping,
 * and aggregation").
 *
 * Problem statement (Section 1): "select A, count(*), sum(X), min(Z), max(Z)
 * ... group by A" over an unsorted input, with duplicate removal as the case
 * without aggregates; the output is sorted on the grouping key (Section 6.1:
 * sorted output is a by-product of the ordered index).
 *
 * Conventions shared by every entry point:
 *  - All column pointers are DEVICE pointers unless stated otherwise.  The
 *    caller owns and allocates every buffer passed in; the library allocates
 *    no device memory.  Host-side bookkeeping uses ordinary host memory.
 *  - The memory budget of the operator (Section 3, Example 1: a per-operator
 *    memory allotment) is the device workspace passed in; the library uses
 *    no other device memory.  Caller-owned input, output and the pinned spill
 *    buffer do not count toward it.
 *  - Temporary storage for runs (Section 3, run generation; Section 4, wide
 *    merging) is a caller-provided pinned host buffer.
 *  - `stream` is a hipStream_t passed as void*.  Every call is synchronous
 *    with respect to the host: it returns after its work on `stream` is done.
 *  - Keys compare as unsigned 64-bit integers; output is ascending by key.
 *    The int64 sum wraps modulo 2^64.  The float64 sum is accumulated in
 *    float64 and is accurate to 1e-12 * (sum of |x|) per group.  Min and max
 *    apply to the int64 value column.
 *  - On error every output count is 0 unless stated otherwise; no exception
 *    crosses the ABI.  A context is used by one host thread at a time;
 *    separate contexts are independent.
 */
#ifndef INSORT_H
#define INSORT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct isa_ctx isa_ctx;
typedef struct isa_server isa_server;

typedef enum {
    ISA_OK = 0,
    ISA_EINVAL = -1,   /* invalid argument (null column for a requested aggregate, ...) */
    ISA_EBUDGET = -2,  /* workspace below isa_min_workspace_bytes */
    ISA_ESPILL = -3,   /* pinned spill buffer too small, or too many runs to merge */
    ISA_ETRUNC = -4,   /* output capacity below the group count; n_groups = required */
    ISA_EDEVICE = -5,  /* HIP runtime error */
    ISA_ENOMEM = -6,   /* host allocation failed, or server workspace cap exceeded */
    ISA_EUNIMPL = -7,
    ISA_EBUSY = -8     /* server: request not finished / no free slot */
} isa_status;

/* Aggregate selection bits.  aggs == 0 is duplicate removal (keys only). */
enum {
    ISA_COUNT = 1u,    /* count(*) per group                      -> output count   */
    ISA_SUM_I64 = 2u,  /* sum of the int64 value, mod 2^64        -> output sum_i64 */
    ISA_SUM_F64 = 4u,  /* sum of the float64 value                -> output sum_f64 */
    ISA_MIN_I64 = 8u,  /* min of the int64 value                  -> output min_i64 */
    ISA_MAX_I64 = 16u  /* max of the int64 value                  -> output max_i64 */
};

/* Input columns (device).  v_i64 is required when any of SUM_I64, MIN_I64,
 * MAX_I64 is requested, v_f64 when SUM_F64 is; otherwise they may be NULL. */
typedef struct {
    const uint64_t* keys;
    const int64_t* v_i64;
    const double* v_f64;
    uint64_t n_rows;
} isa_input;

/* Output columns (device), capacity rows each.  Columns of aggregates that
 * were not requested may be NULL and are not written.  On return n_groups is
 * the number of groups written (or required, with ISA_ETRUNC). */
typedef struct {
    uint64_t* keys;
    uint64_t* count;
    int64_t* sum_i64;
    double* sum_f64;
    int64_t* min_i64;
    int64_t* max_i64;
    uint64_t capacity;
    uint64_t n_groups;
} isa_output;

/* Device workspace: the operator's memory budget, bytes == mem_budget.
 * Must be 256-byte aligned. */
typedef struct {
    void* dev;
    uint64_t bytes;
} isa_workspace;

/* Temporary storage for runs: pinned host memory (hipHostMalloc or a
 * pin_memory tensor).  host_pinned may be NULL when bytes == 0; then any need
 * to spill returns ISA_ESPILL.  Spilled rows never exceed the input rows, so
 * n_rows * isa_state_row_bytes(aggs) bytes always suffice. */
typedef struct {
    void* host_pinned;
    uint64_t bytes;
} isa_spill;

/* Statistics of one call (Section 6 reports spill volume and run counts). */
typedef struct {
    uint64_t runs;            /* sorted runs written to temporary storage         */
    uint64_t spilled_rows;    /* rows written to temporary storage (= rows read back) */
    uint64_t spilled_bytes;
    uint64_t windows;         /* key windows of the wide merge (0 if no merge)    */
    uint64_t batches;         /* input batches absorbed during run generation     */
    uint64_t index_capacity;  /* rows the in-memory index may hold                */
    uint64_t batch_rows;      /* input rows per batch                             */
    uint64_t peak_ws_bytes;   /* workspace bytes actually used                    */
    double t_rungen_ms;       /* wall time of run generation                      */
    double t_merge_ms;        /* wall time of the wide merge and output           */
    double t_plan_ms;         /* host time of the wide merge before its first read */
    uint64_t merge_steps;     /* preliminary merge steps before the wide merge    */
    uint64_t merge_rows;      /* rows those steps wrote to temporary storage      */
    uint64_t resident_capacity; /* hybrid: keys the resident index may hold (else 0) */
    uint64_t run_capacity;    /* keys the run-generation index may hold           */
} isa_stats;

/* Create a context on HIP device `device`.  Returns ISA_EDEVICE if the device
 * is not a usable gfx950 GPU.  *out is set to NULL on error. */
isa_status isa_ctx_create(int device, isa_ctx** out);
void isa_ctx_destroy(isa_ctx* ctx);

/* Bytes of one intermediate (state) row for the given aggregates: key plus
 * partial aggregates (Section 3.3: index and runs share one row format). */
uint64_t isa_state_row_bytes(uint32_t aggs);

/* Smallest workspace isa_group_by accepts for these aggregates. */
uint64_t isa_min_workspace_bytes(uint32_t aggs);

/*
 * Group the input on its key and aggregate (Sections 3 and 4).
 *
 * Run generation consumes the input in batches; each batch is sorted and its
 * duplicate keys collapsed, then absorbed into an ordered in-memory index of
 * unique keys held in the workspace (Section 3.3; Section 6.1: sort the batch,
 * look its distinct keys up in the ordered index).  When the index cannot
 * absorb a batch within its capacity it is written whole, in key order, to the
 * spill buffer as a run (read-sort-write) and a new index starts.  At the end
 * all runs and the last index are combined in a single wide merge step that
 * processes one key window at a time (Section 4) and produces the sorted
 * output.  With no run written the index is the output.
 *
 * stats may be NULL.  Errors: ISA_EINVAL (null ctx/in/out, a missing column,
 * unknown agg bits), ISA_EBUDGET, ISA_ESPILL, ISA_ETRUNC, ISA_EDEVICE.
 */
isa_status isa_group_by(isa_ctx* ctx, const isa_input* in, uint32_t aggs,
                        isa_workspace ws, isa_spill spill, isa_output* out,
                        isa_stats* stats, void* stream);

/*
 * Group on a key of n_cols int64 columns (ascending, lexicographic, each
 * column signed), with offset-value codes deciding the groups (Section 2: the
 * table of offset-value codes and duplicate removal with them; Section 5: a
 * row's columns are compared at most once, N x K column accesses in all).
 * The rows are ordered by a stable radix sort, one column at a time; every
 * row of the sorted stream is then coded against its predecessor: its offset
 * is the number of leading columns equal to the predecessor's, its value the
 * row's value in the first column that differs (the first row: offset 0).  A
 * row starts a group exactly when its offset is below n_cols (a duplicate has
 * offset n_cols), so the in-stream grouping decides each row with one code.
 *
 * key_cols, out_cols: HOST arrays of n_cols device pointers (input columns of
 * n_rows values; output columns of out->capacity values, the group keys in
 * order).  v_i64: the value column (device), required for SUM_I64, MIN_I64,
 * MAX_I64.  aggs: any of ISA_COUNT, ISA_SUM_I64, ISA_MIN_I64, ISA_MAX_I64 (0:
 * duplicate removal); out->keys is unused.  code_offset (uint32) and
 * code_value (int64), both optional device arrays of n_rows entries, receive
 * the sorted stream's codes (code_value is 0 for a duplicate).
 * *column_compares (optional, host) receives the column values compared to
 * code the stream: at most (n_rows - 1) * n_cols.  No spilling: the
 * workspace must hold isa_columns_workspace_bytes(n_rows, n_cols).
 * Errors: ISA_EINVAL (null pointers, n_cols outside 1..ISA_MAX_KEY_COLUMNS,
 * ISA_SUM_F64 requested, n_rows >= 2^32), ISA_EBUDGET, ISA_ETRUNC
 * (out->n_groups = required), ISA_EDEVICE.
 */
enum { ISA_MAX_KEY_COLUMNS = 16 };
isa_status isa_group_by_columns(isa_ctx* ctx, const int64_t* const* key_cols, uint32_t n_cols,
                                const int64_t* v_i64, uint64_t n_rows, uint32_t aggs, isa_workspace ws,
                                int64_t* const* out_cols, isa_output* out, uint32_t* code_offset,
                                int64_t* code_value, uint64_t* column_compares, void* stream);
uint64_t isa_columns_workspace_bytes(uint64_t n_rows, uint32_t n_cols);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * grouping as isa_group_by for an input whose whole sort fits the library's
 * own device scratch, with no workspace argument and no spill.  The scratch is
 * one file-scope device array of 64 MiB per GPU, held until the process ends;
 * its address is looked up once per device by isa_ctx_create.  The call
 * allocates no device or pinned memory and creates no stream, event or graph
 * (the pinned staging and events it uses are set up by isa_ctx_create); were
 * it to need any, it returns ISA_ENOMEM instead.  Results are those of
 * isa_group_by (the same kernels).  Every call on a GPU shares that GPU's
 * scratch: calls that overlap on one GPU (from different contexts, or
 * different streams) race and must be serialised by the caller.
 * Errors: ISA_EBUDGET when in->n_rows > isa_noalloc_max_rows(aggs); otherwise
 * as for isa_group_by (ISA_EINVAL, ISA_ETRUNC, ISA_EDEVICE).
 */
isa_status isa_group_by_noalloc(isa_ctx* ctx, const isa_input* in, uint32_t aggs,
                                isa_output* out, void* stream);
/* Largest n_rows isa_group_by_noalloc accepts for these aggregates
 * (0 for unknown aggregate bits).  Host-only. */
uint64_t isa_noalloc_max_rows(uint32_t aggs);

/*
 * Group input that is already sorted on its key (ascending, unsigned): the
 * in-stream aggregation of the paper's decision table for sorted input (§1,
 * and §2.1 on in-stream grouping) with no sort and no run.  One pass finds the
 * groups, a second reduces them; groups longer than 4096 rows are reduced in
 * parallel pieces.  The workspace holds only per-4096-row bookkeeping (about
 * 48 bytes per 4096 input rows).  Errors: ISA_EINVAL if a key is below its
 * predecessor (nothing is written), ISA_ETRUNC (n_groups = required), as for
 * isa_group_by otherwise.
 */
isa_status isa_group_by_sorted(isa_ctx* ctx, const isa_input* in, uint32_t aggs, isa_workspace ws,
                               isa_output* out, void* stream);

/*
 * count(*) and count(distinct x) grouped by g, from one sort on (g, x): the
 * paper's case for one sort serving duplicate removal and grouping together
 * (§1; §6, Hypothesis 6).  The pair (g, x) of int32 columns becomes one
 * normalized 64-bit key (signed order of g, then of x).  The pairs are grouped
 * with count(*) by the path of isa_group_by (run generation under the budget
 * `ws`, runs spilled to `spill`, wide merge), and the resulting sorted pairs
 * are grouped again on g alone in one in-stream pass (count = sum of the pair
 * counts, distinct = number of pairs).
 * pair_scratch: device memory outside the budget, owned by the caller:
 * 8 bytes per input row plus 16 per distinct pair; 24 * n_rows bytes always
 * suffice.  Output (device, capacity rows): out_g ascending (signed),
 * out_count, out_distinct; *n_groups is set as for isa_group_by.
 * Errors: ISA_EINVAL (null columns), ISA_EBUDGET (workspace below the minimum,
 * or pair_scratch too small for the distinct pairs), ISA_ESPILL, ISA_ETRUNC.
 */
isa_status isa_count_distinct(isa_ctx* ctx, const int32_t* g, const int32_t* x, uint64_t n_rows,
                              isa_workspace ws, isa_spill spill, void* pair_scratch,
                              uint64_t scratch_bytes, int32_t* out_g, uint64_t* out_count,
                              uint64_t* out_distinct, uint64_t capacity, uint64_t* n_groups,
                              void* stream);

/*
 * Group on the pair (a, b) of int32 columns for input sorted on a only
 * (Section 1: with input sorted on a prefix of the grouping key, grouping
 * proceeds one segment at a time).  Each a-segment is grouped on b
 * independently; segments are processed together in waves that fit the
 * workspace, enqueued on the stream one after another (output rows are
 * carried between waves on the device).  Output is
 * ordered by (a, b), both signed, in out_a/out_b (device, capacity rows) and
 * the aggregate columns of out (out->keys is unused and may be NULL).
 * Requires a to be non-decreasing (ISA_EINVAL if a segment boundary check
 * fails).  No spilling: every segment's output must fit the workspace
 * (ISA_EBUDGET otherwise).
 */
isa_status isa_group_by_segmented(isa_ctx* ctx, const int32_t* a_sorted,
                                  const int32_t* b, const int64_t* v,
                                  uint64_t n_rows, uint32_t aggs, isa_workspace ws,
                                  int32_t* out_a, int32_t* out_b, isa_output* out,
                                  void* stream);

/*
 * Run n_inst independent group-by instances together: every phase of the
 * device path is launched once for all instances (the launches can be replayed
 * as one captured graph).  `inst` and `outs` are HOST arrays of n_inst entries
 * whose column pointers are device pointers.  No spilling: all instances'
 * intermediate data must fit the workspace together (ISA_EBUDGET otherwise;
 * isa_batch_workspace_bytes gives the requirement).  On ISA_ETRUNC the
 * failing instances have n_groups = required and the others are complete.
 */
isa_status isa_batch_run(isa_ctx* ctx, uint32_t n_inst, const isa_input* inst,
                         uint32_t aggs, isa_workspace ws, isa_output* outs,
                         void* stream);
uint64_t isa_batch_workspace_bytes(uint32_t n_inst, const isa_input* inst, uint32_t aggs);

/*
 * Run generation policy of isa_group_by when the index fills (Section 3: an
 * ordered in-memory index supports both; the choice is the implementer's).
 *  ISA_RUNGEN_READ_SORT_WRITE (default): the whole index is written as one run
 *    (count-1 rows compacted to raw columns, integer values in 4 bytes when
 *    all of the run's fit) and emptied.
 *  ISA_RUNGEN_REPLACEMENT: replacement selection through the index.  A scan
 *    cursor moves through the index in key order; when an absorbed batch makes
 *    the index exceed its capacity, the excess rows at or after the cursor are
 *    evicted in key order to the open run (state rows); when the scan passes
 *    the largest key the run ends and the scan restarts at the smallest key.
 *    Runs average about twice the index for random input and the whole input
 *    for sorted input.
 * Held per context; ISA_EINVAL for an unknown policy.
 */
enum { ISA_RUNGEN_READ_SORT_WRITE = 0, ISA_RUNGEN_REPLACEMENT = 1, ISA_RUNGEN_HYBRID = 2 };
isa_status isa_set_run_generation(isa_ctx* ctx, int policy);
/*
 * ISA_RUNGEN_HYBRID, hybrid run generation (Section 5, hybrid algorithms):
 * the index memory is divided between a resident index, which removes the
 * duplicates of the key values assigned to it for good, and a run-generation
 * index for the other key values, written as a run whenever it cannot absorb a
 * batch (read-sort-write).  Key values are assigned as the input arrives:
 * keys below a cut stay resident; the cut starts above every key, and when the
 * resident index outgrows its share, its keys beyond the first three quarters
 * of that share are written as one run and the cut moves down to the first
 * of them.  Both indexes join the final wide merge.  isa_set_resident_share
 * sets the resident index's share of the index memory in thousandths
 * (default 800, the share of the paper's example; the run-generation index
 * keeps at least one batch); a share that leaves the resident index smaller
 * than a batch means no resident index.  ISA_EINVAL above 1000.
 */
isa_status isa_set_resident_share(isa_ctx* ctx, uint32_t permille);
int isa_get_run_generation(isa_ctx* ctx); /* the policy, or -1 for a NULL context */

/*
 * Launch configuration of the device plans, held per context: the search
 * space of the autotuner below.  It changes speed only, never results.
 * Defaults: leaf_rows 2048, chunk_split 512, graph 1, merge_fanin 0.
 */
typedef struct {
    uint32_t leaf_rows;    /* target rows per sort leaf (buckets per partition = rows / leaf_rows,
                              2..256); 256..2048 */
    uint32_t chunk_split;  /* partition chunks per region: chunk rows = rows / chunk_split, clamped
                              to 4096..16384 (2048..16384 for the batches of isa_group_by); 64..4096 */
    uint32_t graph;        /* 1: a wave of small batched instances launches as one captured HIP
                              graph; 0: direct launches */
    uint32_t merge_fanin;  /* runs one merge step of isa_group_by may take (Section 4's merge
                              fan-in F): 0 = every run in one wide merge while a window fits
                              the workspace; 2..65536 = when more runs were written, preliminary
                              merge steps of the smallest runs come first (Section 4, Example 4)
                              so that the final wide merge takes at most this many */
} isa_tuning;
isa_status isa_get_tuning(isa_ctx* ctx, isa_tuning* out);
/* ISA_EINVAL when a field is outside its range. */
isa_status isa_set_tuning(isa_ctx* ctx, const isa_tuning* t);

/*
 * Autotuner for batched runs.  Writes the candidate grid (leaf_rows x
 * chunk_split x graph) to out[0..max) and returns its size.
 */
uint32_t isa_tune_candidates(isa_tuning* out, uint32_t max);
/*
 * Runs isa_batch_run on the given instances under every candidate
 * configuration (twice each, keeping the shorter wall time), leaves the
 * fastest configuration set on the context and stores it in *best.  The
 * outputs hold the results of the last run (identical under every
 * configuration).  times_ms (may be NULL) receives each candidate's time in
 * the order of isa_tune_candidates, up to n_times entries.  Errors as for
 * isa_batch_run; on error the context keeps its previous configuration.
 */
isa_status isa_tune_batch(isa_ctx* ctx, uint32_t n_inst, const isa_input* inst, uint32_t aggs,
                          isa_workspace ws, isa_output* outs, void* stream, isa_tuning* best,
                          double* times_ms, uint32_t n_times);

/*
 * Serving: a request loop that admits group-by requests against a device
 * workspace cap and runs admitted requests together (continuous batching):
 * requests that arrive while others run are admitted as soon as workspace and
 * a slot free up, and their device work overlaps.  The server owns a worker
 * thread; hbm_cap_bytes of workspace are carved from `workspace` (device,
 * caller-owned, at least hbm_cap_bytes).  Input and output buffers of a
 * request must stay valid until isa_server_poll reports it done.
 */
isa_status isa_server_create(isa_ctx* ctx, void* workspace, uint64_t hbm_cap_bytes,
                             uint32_t slots, isa_server** out);
/* Enqueue a request; *ticket identifies it.  ISA_ENOMEM if the request alone
 * could never fit the cap. */
isa_status isa_server_submit(isa_server* s, const isa_input* in, uint32_t aggs,
                             isa_output* out, uint64_t* ticket);
/* *done = 1 once the request finished; then *latency_ms is arrival-to-ready
 * time, out->n_groups is set and the return value is the request's status. */
isa_status isa_server_poll(isa_server* s, uint64_t ticket, int* done, double* latency_ms);
/* Forget a finished request: its record is freed and its ticket becomes
 * unknown (a long-lived server calls this once it has read a result).
 * ISA_EBUSY if the request has not finished, ISA_EINVAL for an unknown ticket.
 * The caller's output buffers are untouched. */
isa_status isa_server_release(isa_server* s, uint64_t ticket);
/* Block until every submitted request finished. */
isa_status isa_server_drain(isa_server* s);
void isa_server_destroy(isa_server* s);

const char* isa_status_str(isa_status st);

/* Per-kernel timing of launches on a context (instrumentation for
 * measurement; not part of the grouping semantics).  isa_profile_enable(ctx,1)
 * clears the record and brackets every later kernel launch and host-link copy
 * of the context with HIP events on its stream; 0 stops recording.
 * isa_profile_read aggregates the record by name into out[0..max) and returns
 * the number of distinct names (or a negative isa_status).  `rows` are the
 * units the launches processed, `bytes` their algorithmic bytes (each unit's
 * row read once). */
typedef struct {
    char name[32];
    uint64_t launches;
    uint64_t rows;
    uint64_t bytes;
    double total_ms;
} isa_kernel_time;
isa_status isa_profile_enable(isa_ctx* ctx, int on);
int isa_profile_read(isa_ctx* ctx, isa_kernel_time* out, int max);

/* Message describing the last error returned on this context ("" if none).
 * The string is owned by the context and valid until its next call. */
const char* isa_last_error(isa_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* INSORT_H */
