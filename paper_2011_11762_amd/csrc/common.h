// Internal declarations of libqbsm (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qbsm.h"

namespace qbsm {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
    qbsm_status st;
    Error(qbsm_status s, const std::string &m) : std::runtime_error(m), st(s) {}
};

#define QB_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::qbsm::Error(QBSM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define QB_CHECK(cond, st, msg)                                                           \
    do {                                                                                  \
        if (!(cond)) throw ::qbsm::Error((st), (msg));                                    \
    } while (0)

#define QB_LAUNCH_CHECK() QB_HIP(hipGetLastError())

// --------------------------------------------------------------- allocation
void *dalloc(size_t bytes, hipStream_t s);
void dfree(void *p, hipStream_t s);

// Owning device array; memory is returned on the stream it was taken on.
template <class T>
struct DArr {
    T *p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;

    DArr() = default;
    DArr(size_t count, hipStream_t st) { alloc(count, st); }
    DArr(const DArr &) = delete;
    DArr &operator=(const DArr &) = delete;
    DArr(DArr &&o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
    DArr &operator=(DArr &&o) noexcept {
        if (this != &o) { reset(); p = o.p; n = o.n; s = o.s; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DArr() { reset(); }
    void alloc(size_t count, hipStream_t st) {
        reset();
        s = st;
        n = count;
        p = count ? static_cast<T *>(dalloc(count * sizeof(T), st)) : nullptr;
    }
    void reset() {
        if (p) dfree(p, s);
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
};

// ------------------------------------------------------------ device utils
// Device-wide exclusive scan of int32 counts.  out[0..n] receives the
// exclusive prefix sums followed by the total at out[n]; the 64-bit total is
// also written to *total64 (device).  Throws if the total exceeds INT32_MAX
// only when the caller reads it back; callers check.
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int64_t *total64,
                        hipStream_t s);
// Same for int64 values (no overflow concerns at these sizes).
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
// Tiles of the scans: kScanThreads threads of kScanItems consecutive values.
constexpr int kScanThreads = 256, kScanItems = 8;
constexpr int64_t kScanTile = (int64_t)kScanThreads * kScanItems;
// exclusive_scan_i32 for values whose producer kernel already wrote their
// sums by parts: partial[t] is the sum of [t * kScanTile / sub, (t + 1) *
// kScanTile / sub), sub = 1 or 8 parts per tile; partial holds
// ceil(n * sub / kScanTile) + 1 entries and may be overwritten.  n > 0.
void exclusive_scan_i32_partials(const int32_t *in, int32_t *out, int64_t n, int64_t *partial, int sub,
                                 int64_t *total64, hipStream_t s);

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void fill_bytes_zero(void *p, size_t bytes, hipStream_t s);

// Reads a device value back (synchronises the stream).
template <class T>
T read_back(const T *dev, hipStream_t s) {
    T v{};
    QB_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    QB_HIP(hipStreamSynchronize(s));
    return v;
}

inline int ceil_log2(int64_t x) {
    int d = 0;
    while ((int64_t(1) << d) < x) ++d;
    return d;
}

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 1 << 30) g = 1 << 30;
    return (unsigned)g;
}

// Rank of unique keys via a presence bitmap: for keys < range, writes
// rank[i] = number of keys smaller than key[i].  Duplicate keys set
// *dup_flag (device) to 1.  Keys are uint32.  Returns nothing; the count of
// distinct keys is written to *count (device int64).
void bitmap_rank(const uint32_t *keys, const uint8_t *active, int64_t n, uint64_t range,
                 int32_t *rank, int32_t *dup_flag, int64_t *count, hipStream_t s);

// ----------------------------------------------------------------- handles
enum Storage { ST_NONE = 0, ST_F64 = 1, ST_F32 = 2 };

// Ozaki mode: each element is truncated to an integer M of OZ_MANT bits on
// its line's exponent grid and stored as OZ_SLICES balanced digits of OZ_BITS
// bits (each in [-128, 127], an 8-bit integer); a packed leaf holds the
// slices [slice][chunk][line][bytes] followed by one int32 exponent per
// line.  OZ_MAXM is the largest M the digits reach.  OZ_NONFINITE marks a
// line that holds an Inf or NaN.
constexpr int OZ_SLICES = 6, OZ_BITS = 8, OZ_MANT = 47;
constexpr int64_t OZ_MAXM = 127 * (((int64_t)1 << (OZ_SLICES * OZ_BITS)) - 1) / ((1 << OZ_BITS) - 1);
constexpr int32_t OZ_NONFINITE = 0x10000000;  // twice it still fits an int32
__host__ __device__ constexpr int64_t oz_leaf_bytes(int bs) {
    return (int64_t)OZ_SLICES * bs * bs + 4 * (int64_t)bs;
}
__host__ __device__ inline int32_t *oz_exponents(uint8_t *pack, int64_t leaf, int bs) {
    return reinterpret_cast<int32_t *>(pack + leaf * oz_leaf_bytes(bs) + (int64_t)OZ_SLICES * bs * bs);
}
enum Role { ROLE_ROW = 0, ROLE_COL = 1 };  // lines = rows / lines = columns

// Sparse quadtree of one matrix at a given depth (paper Sec. 2.1: a node
// refers to four children, nil = -1 means an identically zero quadrant).
struct Tree {
    int D = 0;
    std::vector<int64_t> n;               // nodes per level, 0..D
    std::vector<DArr<int32_t>> child;     // levels 0..D-1: [n_l * 4], slot q = 2*rowbit + colbit
    std::vector<DArr<uint32_t>> key;      // levels 0..D: node Morton key at that level
    std::map<int, DArr<int32_t>> desc;    // s -> leaf indices below level D-s nodes [n * 4^s]
};

struct Pack {
    DArr<uint8_t> buf;
    DArr<int32_t> nonfinite;  // [1]: set by the pack kernel when a packed value is Inf or NaN
    uint64_t version = 0;
    // A pack made ahead of use runs on the library's side stream and records
    // this event; until a stream has waited for it, the buffers may still be
    // being written.
    hipEvent_t ready = nullptr;
    Pack() = default;
    Pack(const Pack &) = delete;
    Pack &operator=(const Pack &) = delete;
    ~Pack();
    // Orders s (and the streams the buffers were taken on) after a pending
    // pack, then forgets the event.
    void settle(hipStream_t s);
};

struct Matrix {
    int64_t nrows = 0, ncols = 0;
    int32_t bs = 0;
    int64_t nbr = 0, nbc = 0;
    int64_t nblk = 0;
    bool has_blocks = false;
    DArr<uint32_t> keys;  // Morton keys of the stored blocks, ascending (storage order)
    DArr<double> v64;     // FP64 values [nblk * bs * bs] (storage order, column-major)
    DArr<float> v32;      // FP32 values when the matrix is an FP32 result
    Storage storage = ST_NONE;
    uint64_t version = 0;    // bumped on every value change
    uint64_t filled_by = 0;  // id of the plan that last wrote this matrix as an output
    uint64_t pattern_id = 0; // bumped on every pattern change
    uint64_t storage_id = 0; // bumped whenever the value array is replaced or freed
    DArr<double> norms;      // leaf Frobenius norms, valid when norms_version == version
    uint64_t norms_version = ~0ull;
    std::map<int, std::unique_ptr<Tree>> trees;         // by depth
    std::map<std::pair<int, int>, Pack> packs;          // (mode, role)
    hipStream_t stream = nullptr;                       // stream of the last allocation
};

// Work description of one output (C) quadtree node at the unit level.
struct Plan {
    Matrix *L = nullptr, *R = nullptr, *M = nullptr;
    int transL = 0, transR = 0;
    uint64_t patL = 0, patR = 0, patM = 0;
    int D = 0, s = 0, unit = 0, bs = 0, lpu = 1;
    int64_t out_rows = 0, out_cols = 0;
    int64_t nunits = 0, npairs = 0, nprod = 0, nout = 0, flops = 0;
    double spamm_tol = 0.0;  // > 0: leaf products selected by the norm-product test
    int upper = 0;           // 1: output blocks with I <= J only
    int sched = 0;           // numeric schedule: 0 automatic, 1 one workgroup per unit, 2 streamed
    DArr<int32_t> ustart;   // [nunits + 1] pair range of each unit
    DArr<uint32_t> ukey;    // [nunits] Morton key of the unit node
    DArr<int32_t> umask;    // [nunits] mask-tree node of the unit (masked plans)
    DArr<int32_t> pl, pr;   // [npairs] L / R node indices at the unit level
    DArr<uint64_t> pmask;   // [npairs] leaf-product bits ((kb*lpu + ib)*lpu + jb)
    DArr<int32_t> cdesc;    // [nunits * lpu*lpu] output leaf index, -1 none (row-major ib,jb)
    DArr<uint32_t> okeys;   // [nout] output Morton keys (unmasked plans)
    hipStream_t stream = nullptr;
    uint64_t id = 0;        // process-unique plan id
};

struct Allocator {
    qbsm_alloc_fn alloc = nullptr;
    qbsm_release_fn release = nullptr;
    void *ctx = nullptr;
};
Allocator &allocator();

// -------------------------------------------------------------- operations
int64_t matrix_set_blocks(Matrix &m, int64_t nblk, const int32_t *brow, const int32_t *bcol,
                          const double *vals, double drop_tol, hipStream_t s);
void matrix_store_f32(Matrix &m, hipStream_t s);
Tree &matrix_tree(Matrix &m, int D, hipStream_t s);
const int32_t *tree_desc(Matrix &m, Tree &t, int s_lvl, hipStream_t st);
void matrix_get_pattern(Matrix &m, int32_t *brow, int32_t *bcol, hipStream_t s);
void matrix_get_values(Matrix &m, double *vals, hipStream_t s);
void matrix_extract_blocks(Matrix &m, int64_t n, const int32_t *brow, const int32_t *bcol, double *vals,
                           hipStream_t s);
void matrix_morton_to_rowmajor_rank(Matrix &m, int32_t *rank, hipStream_t s);

// spamm_tol > 0: sparse approximate multiply (leaf products with
// ||L leaf||_F * ||R leaf||_F < spamm_tol are left out).
// upper != 0: only the output blocks with I <= J (square outputs; the
// symmetric square keeps the upper triangle of a symmetric product).
std::unique_ptr<Plan> plan_build(Matrix *L, int transL, Matrix *R, int transR, Matrix *M,
                                 int unit, double spamm_tol, int upper, hipStream_t s);
// FP64 Frobenius norm of every stored leaf (storage order), cached per value version.
const double *matrix_norms(Matrix &m, hipStream_t s);
// Element-level assignment / extraction and error-controlled truncation.
int64_t matrix_set_elements(Matrix &m, int64_t n, const int64_t *row, const int64_t *col, const double *val,
                            hipStream_t s);
void matrix_get_elements(Matrix &m, int64_t n, const int64_t *row, const int64_t *col, double *val,
                         hipStream_t s);
int64_t matrix_truncate(Matrix &m, double eps, hipStream_t s);
void matrix_add(double alpha, Matrix &A, double beta, Matrix &B, Matrix &C, hipStream_t s);
void matrix_add_identity(Matrix &A, double sigma, hipStream_t s);
void plan_get_products(Plan &p, int32_t *I, int32_t *K, int32_t *J, hipStream_t s);
// QBSM_ERR_STATE unless the plan's operands still have their patterns.
void plan_check_current(const Plan &p);
// Masked backward plans regrouped from a forward plan (no symbolic walk):
// which 0 gives dA = (dC op(R)^T) on L's pattern, 1 gives dB = (op(L)^T dC)
// on R's pattern.  The forward plan must be a regular one (no transposes,
// mask, approximation or triangle option).
bool plan_backward_ok(const Plan &f);
std::unique_ptr<Plan> plan_backward(const Plan &f, Matrix *dC, int which, hipStream_t s);

// Packs operand values for (mode, role); returns the device buffer and the
// strides (in elements) the numeric kernel uses to address leaf lines.
struct PackView {
    const void *ptr = nullptr;
    int64_t leaf_stride = 0;  // elements between consecutive leaves
    int64_t part_stride = 0;  // elements between hi and lo parts
    int32_t line_stride = 0;  // elements between consecutive lines of a leaf chunk
    int32_t chunk_stride = 0; // elements between consecutive K chunks
    const int32_t *nonfinite = nullptr;  // device flag of the pack
};
PackView matrix_pack(Matrix &m, qbsm_mode mode, Role role, hipStream_t s);
// Bytes of one (mode, role) pack of m.
size_t pack_bytes(const Matrix &m, qbsm_mode mode);
// Strides of a pack of m for `mode` stored at buf.
PackView pack_view(const Matrix &m, qbsm_mode mode, const void *buf, const int32_t *nonfinite);
// Packs m's current values for (mode, role) into caller-provided device
// memory: dst (pack_bytes) and nonfinite (one int32 flag, cleared first).
// Launches only.
void pack_into(Matrix &m, qbsm_mode mode, Role role, uint8_t *dst, int32_t *nonfinite, hipStream_t s);
// Brings both packs (row and column lines) of m up to date in one pass when
// both are stale; otherwise leaves them to matrix_pack.
void matrix_pack_pair(Matrix &m, qbsm_mode mode, hipStream_t s);
// Packs ahead of use on the side stream (roles: bit 0 row lines, bit 1
// column lines), after the work queued on s; buffers are taken on s.
void matrix_prepack(Matrix &m, qbsm_mode mode, int roles, hipStream_t s);
// Orders s, and the streams of m's value arrays, after every pending pack of
// m; called before m's values or packs are replaced or freed.
void matrix_settle(Matrix &m, hipStream_t s);
// The library's stream for work made ahead of use (one per device, default
// priority, created on first use).
hipStream_t side_stream();
int mode_bk(qbsm_mode mode, int bs);

void numeric_prepare_output(Plan &p, qbsm_mode mode, Matrix &out, hipStream_t s);
// Checks that a plan is still current and runs at unit p.unit in `mode`.
void numeric_check(const Plan &p, qbsm_mode mode);
void numeric_launch(Plan &p, qbsm_mode mode, Matrix &out, hipStream_t s);
// Grid of the streamed numeric schedule for this plan and mode (resident
// workgroups, each running every G-th unit), or 0 for one workgroup per unit.
int numeric_stream_grid(const Plan &p, qbsm_mode mode);

// Kernel-side member description (also used by the batched launch).
struct K5Member {
    const int32_t *ustart;
    const uint32_t *ukey;
    const int32_t *pl;
    const int32_t *pr;
    const uint64_t *pmask;
    const int32_t *descL;  // nullptr: identity (s == 0)
    const int32_t *descR;
    const int32_t *cdesc;
    const void *packL;
    const void *packR;
    void *C;
    int64_t leafStrideL, partStrideL, leafStrideR, partStrideR;
    int32_t lineStrideL, chunkStrideL, lineStrideR, chunkStrideR;
    const int32_t *nfL, *nfR;  // non-finite flags of the two packs (device)
    int64_t out_rows, out_cols;
    int32_t nunits, bs, s, lpu, transL, transR;
    int32_t select;  // 1: leaf products chosen one by one (sparse approximate multiply)
    int32_t pad1;
};

struct Batch {
    int32_t n = 0;
    qbsm_mode mode = QBSM_F64;
    int unit = 0;
    std::vector<Plan *> plans;
    std::vector<Matrix *> outs;
    DArr<K5Member> members;
    DArr<int2> items;        // (member, unit) in LPT order
    DArr<int32_t> counter;   // work counter of the persistent launch
    int64_t nitems = 0;
    int wg_per_cu = 0;
    int num_cus = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
    // packing jobs replayed on every run
    // buf / bytes: the pack buffer the member records point to; out_vals /
    // out_pattern: each output's value buffer and pattern id.  A run checks
    // that all are still in place.
    // storage: the operand's storage_id at creation (the captured pack
    // kernels read its value array of that time)
    struct PackJob { Matrix *m; qbsm_mode mode; Role role; const void *buf; size_t bytes; uint64_t storage; };
    std::vector<PackJob> packs;
    std::vector<const void *> out_vals;
    std::vector<uint64_t> out_pattern;
};

K5Member member_from_views(const Plan &p, const int32_t *descL, const int32_t *descR, const PackView &vL,
                           const PackView &vR, void *C);

void batch_init(Batch &b, const std::vector<Plan *> &plans, const std::vector<Matrix *> &outs, qbsm_mode mode,
                hipStream_t s);
void batch_launch(Batch &b, hipStream_t s);
// Checks that the batch's plans, packs and outputs are still the ones its
// member records point to (QBSM_ERR_STATE otherwise), then orders s after
// pending packs of its operands (call outside capture).
void batch_settle(Batch &b, hipStream_t s);
void pack_launch(Matrix &m, qbsm_mode mode, Role role, Pack &pk, hipStream_t s);
// persistent: 0 = one workgroup per unit of `single` (grid = its units);
// 1 = the work list of `members` / `items`; 2 = the streamed schedule of
// `single` (grid = resident workgroups); 3 = one workgroup per unit on the
// single-stage kernel (BF16 modes and FP64 at unit 128).
void k5_launch(qbsm_mode mode, int unit, const K5Member *members, int32_t nmembers_host_unused,
               const int2 *items, int64_t nitems, int32_t *counter, int grid, int persistent,
               const K5Member &single, hipStream_t s);

int device_cu_count();
// Text returned by qbsm_last_error() on this thread.
void set_last_error(const char *msg);

// Optional event timing around kernel launches (kernel classes below).
enum ProfClass { PROF_NUMERIC = 0, PROF_PACK = 1, PROF_NCLASS = 2 };
struct ProfScope {
    int cls;
    hipStream_t s;
    hipEvent_t e1 = nullptr;
    ProfScope(int c, hipStream_t st);
    ~ProfScope();
};

}  // namespace qbsm

// Opaque handles of the C ABI.
struct qbsm_matrix_ {
    qbsm::Matrix m;
};
struct qbsm_plan_ {
    std::unique_ptr<qbsm::Plan> p;
};
struct qbsm_batch_ {
    qbsm::Batch b;
};
