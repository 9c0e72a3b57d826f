// Internal types shared by the host engine and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isa {

// Rows per leaf: the largest key range a single workgroup sorts and reduces
// in LDS (256 threads x 16 rows).
constexpr int LEAF_NT = 256;
constexpr int LEAF_IPT = 16;
constexpr int LEAF_CAP = LEAF_NT * LEAF_IPT;
// Rows per partition chunk (one workgroup of the histogram / scatter passes).
constexpr int PART_NT = 256;
constexpr int PART_IPT = 16;
constexpr int PART_TILE = PART_NT * PART_IPT;
constexpr int PART_CHUNK = 4 * PART_TILE;
// smallest partition chunk (one workgroup's rows): a 524288-row batch spans
// 256 chunks, one per compute unit
constexpr int PART_CHUNK_MIN = PART_TILE / 2;
// Buckets per partition level (8-bit digit of the splitter rank).
constexpr int MAX_BUCKETS = 256;
// Keys sampled per region to choose its splitters.
constexpr int SAMPLE_N = 4096;
// Diagonal length handled by one workgroup of the merge-path merge.
constexpr int MERGE_D = 4096;
// Rows reduced per workgroup for single-key buckets.
constexpr int SINGLE_CHUNK = 4096;

// Strided view of rows: element i of a column lives at col[i * stride].
// Raw input rows have cnt == nullptr (count 1 per row) and sum == mn == mx ==
// the int64 value column.  Absent aggregate columns are nullptr.
struct ColView {
    const uint64_t* key;
    const uint64_t* cnt;
    const int64_t* sum;
    const int64_t* mn;
    const int64_t* mx;
    const double* fs;
    uint64_t stride;
};

// Writable strided view of state rows (key + partial aggregates).
struct OutView {
    uint64_t* key;
    uint64_t* cnt;
    int64_t* sum;
    int64_t* mn;
    int64_t* mx;
    double* fs;
    uint64_t stride;
};

// Row-major layout of rows in partition buffers and of state rows in the
// index and in runs: word offsets (8-byte words), -1 when absent.
struct Layout {
    int32_t words;
    int32_t cnt, sum, mn, mx, fs;
};

// Compact run format, count-1 part: n rows of raw layout R stored column by
// column (keys, then the f64 values when R has them, then the integer values
// when R has them, 4 bytes each when every value of the run fits in 32 bits,
// else 8), padded to a multiple of 8 bytes.
__host__ __device__ inline uint64_t single_bytes(uint64_t n, const Layout& R, bool narrow) {
    uint64_t b = n * 8;
    if (R.fs >= 0) b += n * 8;
    if (R.sum >= 0) b += n * (narrow ? 4 : 8);
    return (b + 7) & ~7ull;
}

// Compact run format, packed part: the rows of count above 1 whose count
// fits in 32 bits and whose integer sum, min and max fit in 32-bit signed
// values, each as the key, the f64 sum (when present) and then the 32-bit
// fields count, sum, min, max (those present), two to a word, low half first.
// Used when narrower than a state row (packed_words(S) < S.words).
__host__ __device__ inline int packed_words(const Layout& S) {
    const int nf = (S.cnt >= 0 ? 1 : 0) + (S.sum >= 0 ? 3 : 0);
    return 1 + (S.fs >= 0 ? 1 : 0) + (nf + 1) / 2;
}
__host__ __device__ inline bool has_packed(const Layout& S) { return S.cnt >= 0 && packed_words(S) < S.words; }
// Bytes of a compact run: its count-1 part, packed part and state rows.
__host__ __device__ inline uint64_t compact_bytes(uint64_t n_single, uint64_t n_packed, uint64_t n_state,
                                                  const Layout& R, const Layout& S, bool narrow) {
    return single_bytes(n_single, R, narrow) + (n_packed * (uint64_t)packed_words(S) + n_state * (uint64_t)S.words) * 8;
}

// One region being partitioned at the current level.
struct Region {
    ColView src;        // its rows are src[0, n)
    uint64_t n;
    uint64_t out_pos;   // first row of the region in the target partition buffer
    uint64_t hist_base; // offset of its nb x n_chunks histogram (bucket-major)
    uint32_t nb;        // buckets, 2..MAX_BUCKETS
    uint32_t n_chunks;
};

// One workgroup's share of a region in the histogram and scatter passes.
struct Chunk {
    uint32_t region;
    uint32_t idx;       // chunk index within the region
    uint64_t start;     // first row within the region
    uint32_t n;
    uint32_t pad;
};

// A key range small enough to sort and reduce in one workgroup (kind 0), or
// a range holding a single key value of any size (kind 1).
struct Leaf {
    ColView src;
    uint64_t n;
    uint64_t out_pos;   // first row of its (gapped) output in the temp buffer
    uint32_t kind;
    uint32_t single_first;  // kind 1: first partial slot
    uint32_t single_count;  // kind 1: number of partials
    uint32_t pad;
};

// A piece of a single-key leaf reduced by one workgroup into one partial.
struct SinglePiece {
    uint32_t leaf;
    uint32_t slot;
    uint64_t start;
    uint32_t n;
    uint32_t pad;
};

// Largest instance the single-level flat plan takes: every bucket of a full
// 256-way split then averages half a leaf.
constexpr uint64_t FLAT_MAX = (uint64_t)LEAF_CAP * MAX_BUCKETS / 2;

// One leaf slot of the flat plan: a whole small instance (kind 0) or one
// bucket of a partitioned instance (kind 1).
struct FlatSlot {
    uint32_t kind;
    uint32_t idx;     // instance index (kind 0) or region index (kind 1)
    uint32_t bucket;
    uint32_t dest;
};

struct FlatInst {
    ColView src;
    uint64_t n;
};

// Bytes of the library-owned device scratch used by the entry point for
// callers that cannot allocate (one copy per GPU).
constexpr uint64_t NOALLOC_SCRATCH_BYTES = 64ull << 20;

// Destination of one instance's sorted unique output.
struct Dest {
    OutView out;
    uint64_t capacity;
    // rows already in the destination, read on the device when the leaves
    // start (the end row an earlier launch wrote); nullptr means none
    const uint64_t* base = nullptr;
    // nonzero: the key column is a buffer of this launch's own, indexed from
    // the base row (its row 0 is the destination's row *base); the other
    // columns are the destination's
    uint64_t key_local = 0;
};

// Rows per gather task of the wide merge (a raw slice is staged in LDS).
constexpr uint32_t GATHER_ROWS = 1024;

// One slice of a wide-merge window copied into the window's staging buffer.
struct GatherTask {
    const uint64_t* src;  // first row (state rows) or first key (count-1 rows):
                          // host-mapped pinned memory or device memory
    const uint64_t* fv;   // count-1 rows: their f64 values (when present)
    const void* iv;       // count-1 rows: their integer values (when present)
    uint64_t dst_row;     // first state row written in the staging buffer
    uint32_t n;           // rows, at most GATHER_ROWS
    uint32_t raw;         // 0: state rows; count-1 rows, expanded to state rows,
                          // with 8-byte (1) or 4-byte (2) integer values;
                          // 3: packed rows (packed_words), expanded
};

// A span of gapped output copied into its final place.
struct Segment {
    uint64_t src_pos;
    uint32_t inst;
    uint32_t pad;
};

}  // namespace isa
