// The C ABI of libqbsm: argument checks, error mapping, handle lifetimes,
// batched launches with HIP graph replay, and the unit-size autotuner.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

#include "common.h"

namespace qbsm {

K5Member make_member(Plan &p, qbsm_mode mode, Matrix &out, hipStream_t s);
int k5_occupancy(qbsm_mode mode, int unit, int bs);

namespace {
thread_local std::string g_last_error;

Allocator g_alloc;
}  // namespace

Allocator &allocator() { return g_alloc; }

void set_last_error(const char *msg) { g_last_error = msg; }

namespace {
// Without a hook, memory comes from the device's default stream-ordered pool.
// Its release threshold is raised once per device so that the temporaries a
// call frees stay in the pool for the next call instead of going back to the
// driver at every synchronisation.
std::atomic<bool> g_pool_tuned[64];

void keep_pool_memory() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    if (g_pool_tuned[dev].load(std::memory_order_acquire)) return;
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    g_pool_tuned[dev].store(true, std::memory_order_release);
}
}  // namespace

namespace {
void *raw_alloc(size_t bytes, hipStream_t s) {
    void *p = nullptr;
    if (g_alloc.alloc) {
        p = g_alloc.alloc(bytes, (void *)s, g_alloc.ctx);
    } else {
        keep_pool_memory();
        hipError_t e = hipMallocAsync(&p, bytes, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
    }
    return p;
}

void raw_free(void *p, hipStream_t s) {
    if (g_alloc.release)
        g_alloc.release(p, (void *)s, g_alloc.ctx);
    else
        (void)hipFreeAsync(p, s);
}

// Small temporaries (the symbolic phase takes and returns dozens per call)
// are kept for reuse instead of going back to the allocator, which may be a
// call into another runtime: power-of-two size classes up to 1 MiB, one free
// list per class.  Only blocks of the null stream are cached: it lives as long
// as the process, and a block freed on it is only handed out again on it, so
// stream order covers its last use (a user stream could be destroyed and its
// handle reused).  At most kSmallCacheBytes stay cached; qbsm_set_allocator
// returns them to the allocator they came from first.
constexpr size_t kSmallMax = size_t(1) << 20, kSmallMin = 256, kSmallCacheBytes = size_t(256) << 20;
struct SmallCache {
    std::mutex mu;
    std::map<std::pair<hipStream_t, size_t>, std::vector<void *>> free;
    std::map<void *, size_t> live;  // cached-class blocks handed out: size class
    size_t cached = 0;
};
SmallCache g_small;

size_t small_class(size_t bytes) {
    size_t c = kSmallMin;
    while (c < bytes) c <<= 1;
    return c;
}

void small_trim() {
    std::lock_guard<std::mutex> lock(g_small.mu);
    for (auto &kv : g_small.free)
        for (void *p : kv.second) raw_free(p, kv.first.first);
    g_small.free.clear();
    g_small.cached = 0;
}
}  // namespace

void *dalloc(size_t bytes, hipStream_t s) {
    if (!bytes) return nullptr;
    void *p = nullptr;
    if (bytes <= kSmallMax && s == nullptr) {
        const size_t c = small_class(bytes);
        std::lock_guard<std::mutex> lock(g_small.mu);
        auto it = g_small.free.find({s, c});
        if (it != g_small.free.end() && !it->second.empty()) {
            p = it->second.back();
            it->second.pop_back();
            g_small.cached -= c;
        } else {
            p = raw_alloc(c, s);
        }
        if (p) g_small.live[p] = c;
    } else {
        p = raw_alloc(bytes, s);
    }
    if (!p) throw Error(QBSM_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void dfree(void *p, hipStream_t s) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> lock(g_small.mu);
        auto it = g_small.live.find(p);
        if (it != g_small.live.end()) {
            const size_t c = it->second;
            g_small.live.erase(it);
            if (g_small.cached + c <= kSmallCacheBytes) {
                g_small.free[{s, c}].push_back(p);
                g_small.cached += c;
                return;
            }
        }
    }
    raw_free(p, s);
}

int device_cu_count() {
    int dev = 0;
    QB_HIP(hipGetDevice(&dev));
    int n = 0;
    QB_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    return n;
}

namespace {
struct ProfState {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[PROF_NCLASS];
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
};
ProfState g_prof;
}  // namespace

ProfScope::ProfScope(int c, hipStream_t st) : cls(c), s(st) {
    if (!g_prof.on) return;
    hipEvent_t e0 = g_prof.get();
    e1 = g_prof.get();
    if (!e0 || !e1) { e1 = nullptr; return; }
    (void)hipEventRecord(e0, s);
    g_prof.ev[cls].push_back({e0, e1});
}

ProfScope::~ProfScope() {
    if (e1) (void)hipEventRecord(e1, s);
}

// dA = (dC B^T) on A's pattern and dB = (A^T dC) on B's pattern from the
// forward plan of A * B (either output may be null).
void backward_from(const Plan &f, Matrix &dC, qbsm_mode mode, Matrix *dA, Matrix *dB, hipStream_t s) {
    QB_CHECK(dC.nrows == f.out_rows && dC.ncols == f.out_cols, QBSM_ERR_SHAPE, "dC shape differs from A*B");
    QB_CHECK(dA != &dC && dB != &dC && (!dA || dA != dB), QBSM_ERR_ARG, "outputs alias dC or each other");
    Matrix *outs[2] = {dA, dB};
    for (int which = 0; which < 2; ++which) {
        if (!outs[which]) continue;
        auto p = plan_backward(f, &dC, which, s);
        numeric_prepare_output(*p, mode, *outs[which], s);
        numeric_launch(*p, mode, *outs[which], s);
    }
}

// Everything a batch run needs that allocates or synchronises: outputs,
// operand packs, the member table and the longest-processing-time-first
// work list (the cost of a unit is its number of node pairs).
void batch_init(Batch &b, const std::vector<Plan *> &plans, const std::vector<Matrix *> &outs, qbsm_mode mode,
                hipStream_t s) {
    const int n = (int)plans.size();
    b.n = n;
    b.mode = mode;
    b.num_cus = device_cu_count();
    std::vector<K5Member> hm(n);
    std::vector<std::vector<int32_t>> cost(n);
    for (int i = 0; i < n; ++i) {
        Plan &p = *plans[i];
        if (i == 0) b.unit = p.unit;
        QB_CHECK(p.unit == b.unit, QBSM_ERR_UNSUPPORTED, "all members must use the same unit side");
        for (int j = 0; j < i; ++j) QB_CHECK(outs[j] != outs[i], QBSM_ERR_ARG, "two members share an output");
        numeric_prepare_output(p, mode, *outs[i], s);
        hm[i] = make_member(p, mode, *outs[i], s);
        b.plans.push_back(&p);
        b.outs.push_back(outs[i]);
        b.out_vals.push_back(outs[i]->storage == ST_F64 ? (const void *)outs[i]->v64.p : (const void *)outs[i]->v32.p);
        b.out_pattern.push_back(outs[i]->pattern_id);
        // operand packs replayed on each run
        for (int side = 0; side < 2; ++side) {
            Matrix *mm = side == 0 ? p.L : p.R;
            Role role = side == 0 ? (p.transL ? ROLE_COL : ROLE_ROW) : (p.transR ? ROLE_ROW : ROLE_COL);
            bool seen = false;
            for (auto &j : b.packs) seen |= (j.m == mm && j.mode == mode && j.role == role);
            if (!seen) {
                const Pack &pk = mm->packs[std::make_pair((int)mode, (int)role)];
                b.packs.push_back({mm, mode, role, pk.buf.p, pk.buf.n, mm->storage_id});
            }
        }
        // per-unit cost: number of node pairs (read back for ordering)
        std::vector<int32_t> us(p.nunits + 1);
        if (p.nunits)
            QB_HIP(hipMemcpyAsync(us.data(), p.ustart.p, (p.nunits + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        QB_HIP(hipStreamSynchronize(s));
        cost[i].resize(p.nunits);
        for (int64_t u = 0; u < p.nunits; ++u) cost[i][u] = us[u + 1] - us[u];
    }
    // longest-processing-time-first order over all (member, unit) items
    std::vector<int2> items;
    for (int i = 0; i < n; ++i)
        for (int64_t u = 0; u < (int64_t)cost[i].size(); ++u) items.push_back(make_int2(i, (int)u));
    std::stable_sort(items.begin(), items.end(),
                     [&](const int2 &x, const int2 &y) { return cost[x.x][x.y] > cost[y.x][y.y]; });
    b.nitems = (int64_t)items.size();
    b.members.alloc(n ? n : 1, s);
    b.items.alloc(items.empty() ? 1 : items.size(), s);
    b.counter.alloc(1, s);
    if (n) QB_HIP(hipMemcpyAsync(b.members.p, hm.data(), n * sizeof(K5Member), hipMemcpyHostToDevice, s));
    if (!items.empty())
        QB_HIP(hipMemcpyAsync(b.items.p, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    QB_HIP(hipStreamSynchronize(s));
    b.wg_per_cu = b.unit ? k5_occupancy(mode, b.unit, 0) : 1;
}

}  // namespace qbsm

using namespace qbsm;

namespace {

template <class F>
qbsm_status guard(F &&f) {
    try {
        f();
        return QBSM_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.st;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return QBSM_ERR_OOM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return QBSM_ERR_HIP;
    } catch (...) {
        g_last_error = "unknown failure";
        return QBSM_ERR_HIP;
    }
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

static_assert(sizeof(qbsm_plan_opts) == 32 && offsetof(qbsm_plan_opts, upper) == 4 &&
                  offsetof(qbsm_plan_opts, spamm_tol) == 8,
              "plan options layout is part of the ABI");

bool valid_mode(qbsm_mode m) {
    return m == QBSM_F64 || m == QBSM_F32 || m == QBSM_BF16 || m == QBSM_BF16X3 || m == QBSM_OZAKI_I8;
}

}  // namespace

extern "C" {

qbsm_status qbsm_set_allocator(qbsm_alloc_fn alloc, qbsm_release_fn release, void *ctx) {
    return guard([&] {
        QB_CHECK((alloc == nullptr) == (release == nullptr), QBSM_ERR_ARG, "set both hooks or neither");
        small_trim();  // cached blocks go back to the allocator they came from
        g_alloc.alloc = alloc;
        g_alloc.release = release;
        g_alloc.ctx = ctx;
    });
}

const char *qbsm_status_string(qbsm_status st) {
    switch (st) {
        case QBSM_OK: return "ok";
        case QBSM_ERR_ARG: return "invalid argument";
        case QBSM_ERR_SHAPE: return "shape mismatch";
        case QBSM_ERR_PATTERN: return "invalid block pattern";
        case QBSM_ERR_OOM: return "out of device memory";
        case QBSM_ERR_HIP: return "HIP runtime error";
        case QBSM_ERR_UNSUPPORTED: return "unsupported";
        case QBSM_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

const char *qbsm_last_error(void) { return g_last_error.c_str(); }

int32_t qbsm_version(void) { return 10000; }

qbsm_status qbsm_matrix_create(int64_t nrows, int64_t ncols, int32_t bs, qbsm_matrix *out) {
    return guard([&] {
        QB_CHECK(out, QBSM_ERR_ARG, "null output handle");
        QB_CHECK(nrows >= 0 && ncols >= 0, QBSM_ERR_ARG, "negative size");
        QB_CHECK(bs == 32 || bs == 64 || bs == 128, QBSM_ERR_UNSUPPORTED, "leaf size must be 32, 64 or 128");
        const int64_t nbr = (nrows + bs - 1) / bs, nbc = (ncols + bs - 1) / bs;
        QB_CHECK(nbr <= 65536 && nbc <= 65536, QBSM_ERR_UNSUPPORTED, "block grid side above 65536");
        auto h = std::make_unique<qbsm_matrix_>();
        h->m.nrows = nrows;
        h->m.ncols = ncols;
        h->m.bs = bs;
        h->m.nbr = nbr;
        h->m.nbc = nbc;
        *out = h.release();
    });
}

qbsm_status qbsm_matrix_destroy(qbsm_matrix m) {
    return guard([&] {
        if (m) matrix_settle(m->m, m->m.v64.p ? m->m.v64.s : m->m.v32.s);
        delete m;
    });
}

qbsm_status qbsm_matrix_set_blocks(qbsm_matrix m, int64_t nblk, const int32_t *brow, const int32_t *bcol,
                                   const double *vals, double drop_tol, void *stream, int64_t *nkept) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        const int64_t k = matrix_set_blocks(m->m, nblk, brow, bcol, vals, drop_tol, as_stream(stream));
        if (nkept) *nkept = k;
    });
}

qbsm_status qbsm_matrix_store_f32(qbsm_matrix m, void *stream) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        QB_CHECK(m->m.has_blocks, QBSM_ERR_STATE, "matrix has no blocks yet");
        matrix_store_f32(m->m, as_stream(stream));
    });
}

qbsm_status qbsm_matrix_set_elements(qbsm_matrix m, int64_t n, const int64_t *row, const int64_t *col,
                                     const double *val, void *stream, int64_t *nblk) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        const int64_t k = matrix_set_elements(m->m, n, row, col, val, as_stream(stream));
        if (nblk) *nblk = k;
    });
}

qbsm_status qbsm_matrix_get_elements(qbsm_matrix m, int64_t n, const int64_t *row, const int64_t *col,
                                     double *val, void *stream) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        matrix_get_elements(m->m, n, row, col, val, as_stream(stream));
    });
}

qbsm_status qbsm_matrix_truncate(qbsm_matrix m, double eps, void *stream, int64_t *nkept) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        const int64_t k = matrix_truncate(m->m, eps, as_stream(stream));
        if (nkept) *nkept = k;
    });
}

qbsm_status qbsm_matrix_add(double alpha, qbsm_matrix A, double beta, qbsm_matrix B, qbsm_matrix C,
                            void *stream) {
    return guard([&] {
        QB_CHECK(A && B && C, QBSM_ERR_ARG, "null matrix");
        matrix_add(alpha, A->m, beta, B->m, C->m, as_stream(stream));
    });
}

qbsm_status qbsm_matrix_add_identity(qbsm_matrix A, double sigma, void *stream) {
    return guard([&] {
        QB_CHECK(A, QBSM_ERR_ARG, "null matrix");
        matrix_add_identity(A->m, sigma, as_stream(stream));
    });
}

qbsm_status qbsm_matrix_prepack(qbsm_matrix m, qbsm_mode mode, int32_t roles, void *stream) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        QB_CHECK(valid_mode(mode), QBSM_ERR_ARG, "unknown mode");
        matrix_prepack(m->m, mode, roles, as_stream(stream));
    });
}

qbsm_status qbsm_matrix_info(qbsm_matrix m, int64_t *nrows, int64_t *ncols, int32_t *bs, int64_t *nblk) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        if (nrows) *nrows = m->m.nrows;
        if (ncols) *ncols = m->m.ncols;
        if (bs) *bs = m->m.bs;
        if (nblk) *nblk = m->m.nblk;
    });
}

qbsm_status qbsm_matrix_get_pattern(qbsm_matrix m, int32_t *brow, int32_t *bcol, void *stream) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        QB_CHECK(m->m.nblk == 0 || (brow && bcol), QBSM_ERR_ARG, "null output arrays");
        matrix_get_pattern(m->m, brow, bcol, as_stream(stream));
    });
}

qbsm_status qbsm_matrix_get_values(qbsm_matrix m, double *vals, void *stream) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        QB_CHECK(m->m.nblk == 0 || vals, QBSM_ERR_ARG, "null output array");
        matrix_get_values(m->m, vals, as_stream(stream));
    });
}

qbsm_status qbsm_matrix_extract_blocks(qbsm_matrix m, int64_t n, const int32_t *brow, const int32_t *bcol,
                                       double *vals, void *stream) {
    return guard([&] {
        QB_CHECK(m, QBSM_ERR_ARG, "null matrix");
        matrix_extract_blocks(m->m, n, brow, bcol, vals, as_stream(stream));
    });
}

qbsm_status qbsm_multiply_symbolic_ex(qbsm_matrix L, int32_t trans_l, qbsm_matrix R, int32_t trans_r,
                                      qbsm_matrix mask, const qbsm_plan_opts *opts, void *stream,
                                      qbsm_plan *plan, int64_t *nblk_out, int64_t *nprod) {
    return guard([&] {
        QB_CHECK(L && R && plan, QBSM_ERR_ARG, "null argument");
        const int unit = opts ? opts->unit : 0;
        const double tau = opts ? opts->spamm_tol : 0.0;
        QB_CHECK(tau >= 0.0 && std::isfinite(tau), QBSM_ERR_ARG, "spamm_tol must be finite and >= 0");
        const int upper = opts ? opts->upper : 0;
        QB_CHECK(upper == 0 || upper == 1, QBSM_ERR_ARG, "upper must be 0 or 1");
        const int sched = opts ? opts->schedule : 0;
        QB_CHECK(sched >= 0 && sched <= 2, QBSM_ERR_ARG, "schedule must be 0, 1 or 2");
        if (upper) {
            const int64_t rows = trans_l ? L->m.ncols : L->m.nrows, cols = trans_r ? R->m.nrows : R->m.ncols;
            QB_CHECK(rows == cols, QBSM_ERR_SHAPE, "the upper triangle needs a square product");
            QB_CHECK(!mask, QBSM_ERR_ARG, "upper and a mask do not combine");
        }
        auto p = plan_build(&L->m, trans_l ? 1 : 0, &R->m, trans_r ? 1 : 0, mask ? &mask->m : nullptr, unit, tau,
                            upper, as_stream(stream));
        p->sched = sched;
        if (nblk_out) *nblk_out = p->nout;
        if (nprod) *nprod = p->nprod;
        auto h = std::make_unique<qbsm_plan_>();
        h->p = std::move(p);
        *plan = h.release();
    });
}

qbsm_status qbsm_multiply_symbolic(qbsm_matrix A, qbsm_matrix B, const qbsm_plan_opts *opts, void *stream,
                                   qbsm_plan *plan, int64_t *nblk_C, int64_t *nprod) {
    return qbsm_multiply_symbolic_ex(A, 0, B, 0, nullptr, opts, stream, plan, nblk_C, nprod);
}

qbsm_status qbsm_plan_info(qbsm_plan p, int64_t *nblk_out, int64_t *nprod, int64_t *flops, int32_t *unit,
                           int64_t *nunits, int64_t *npairs) {
    return guard([&] {
        QB_CHECK(p && p->p, QBSM_ERR_ARG, "null plan");
        if (nblk_out) *nblk_out = p->p->nout;
        if (nprod) *nprod = p->p->nprod;
        if (flops) *flops = p->p->flops;
        if (unit) *unit = p->p->unit;
        if (nunits) *nunits = p->p->nunits;
        if (npairs) *npairs = p->p->npairs;
    });
}

qbsm_status qbsm_plan_get_products(qbsm_plan p, int32_t *I, int32_t *K, int32_t *J, void *stream) {
    return guard([&] {
        QB_CHECK(p && p->p, QBSM_ERR_ARG, "null plan");
        QB_CHECK(p->p->nprod == 0 || (I && K && J), QBSM_ERR_ARG, "null output arrays");
        plan_get_products(*p->p, I, K, J, as_stream(stream));
    });
}

qbsm_status qbsm_plan_destroy(qbsm_plan p) {
    return guard([&] { delete p; });
}

qbsm_status qbsm_multiply_numeric(qbsm_plan p, qbsm_mode mode, qbsm_matrix out, void *stream) {
    return guard([&] {
        QB_CHECK(p && p->p && out, QBSM_ERR_ARG, "null argument");
        QB_CHECK(valid_mode(mode), QBSM_ERR_ARG, "unknown mode");
        numeric_prepare_output(*p->p, mode, out->m, as_stream(stream));
        numeric_launch(*p->p, mode, out->m, as_stream(stream));
    });
}

qbsm_status qbsm_multiply_backward(qbsm_matrix A, qbsm_matrix B, qbsm_matrix dC, qbsm_mode mode,
                                   const qbsm_plan_opts *opts, qbsm_matrix dA, qbsm_matrix dB, void *stream) {
    return guard([&] {
        QB_CHECK(A && B && dC, QBSM_ERR_ARG, "null argument");
        QB_CHECK(valid_mode(mode), QBSM_ERR_ARG, "unknown mode");
        QB_CHECK(dC->m.nrows == A->m.nrows && dC->m.ncols == B->m.ncols, QBSM_ERR_SHAPE,
                 "dC shape differs from A*B");
        const int unit = opts ? opts->unit : 0;
        const int sched = opts ? opts->schedule : 0;
        QB_CHECK(sched >= 0 && sched <= 2, QBSM_ERR_ARG, "schedule must be 0, 1 or 2");
        hipStream_t s = as_stream(stream);
        // one symbolic walk for the forward product list, regrouped for both adjoints
        auto f = plan_build(&A->m, 0, &B->m, 0, nullptr, unit, 0.0, 0, s);
        f->sched = sched;
        backward_from(*f, dC->m, mode, dA ? &dA->m : nullptr, dB ? &dB->m : nullptr, s);
    });
}

qbsm_status qbsm_multiply_backward_plan(qbsm_plan forward, qbsm_matrix dC, qbsm_mode mode, qbsm_matrix dA,
                                        qbsm_matrix dB, void *stream) {
    return guard([&] {
        QB_CHECK(forward && forward->p && dC, QBSM_ERR_ARG, "null argument");
        QB_CHECK(valid_mode(mode), QBSM_ERR_ARG, "unknown mode");
        backward_from(*forward->p, dC->m, mode, dA ? &dA->m : nullptr, dB ? &dB->m : nullptr, as_stream(stream));
    });
}

qbsm_status qbsm_batch_create(int32_t n, const qbsm_plan *plans, qbsm_mode mode, qbsm_matrix *outs, void *stream,
                              qbsm_batch *batch) {
    return guard([&] {
        QB_CHECK(n >= 0 && batch && (n == 0 || (plans && outs)), QBSM_ERR_ARG, "null argument");
        QB_CHECK(valid_mode(mode), QBSM_ERR_ARG, "unknown mode");
        std::vector<Plan *> ps(n);
        std::vector<Matrix *> os(n);
        for (int i = 0; i < n; ++i) {
            QB_CHECK(plans[i] && plans[i]->p && outs[i], QBSM_ERR_ARG, "null plan or output");
            ps[i] = plans[i]->p.get();
            os[i] = &outs[i]->m;
        }
        auto h = std::make_unique<qbsm_batch_>();
        batch_init(h->b, ps, os, mode, as_stream(stream));
        *batch = h.release();
    });
}

qbsm_status qbsm_batch_set_occupancy(qbsm_batch batch, int32_t wg_per_cu) {
    return guard([&] {
        QB_CHECK(batch && wg_per_cu >= 0, QBSM_ERR_ARG, "bad argument");
        Batch &b = batch->b;
        b.wg_per_cu = wg_per_cu ? wg_per_cu : (b.unit ? k5_occupancy(b.mode, b.unit, 0) : 1);
        if (b.exec) {
            (void)hipGraphExecDestroy(b.exec);
            (void)hipGraphDestroy(b.graph);
            b.exec = nullptr;
            b.graph = nullptr;
        }
    });
}

qbsm_status qbsm_batch_run(qbsm_batch batch, void *stream) {
    return guard([&] {
        QB_CHECK(batch, QBSM_ERR_ARG, "null batch");
        batch_settle(batch->b, as_stream(stream));
        batch_launch(batch->b, as_stream(stream));
    });
}

qbsm_status qbsm_batch_run_graph(qbsm_batch batch, void *stream) {
    return guard([&] {
        QB_CHECK(batch, QBSM_ERR_ARG, "null batch");
        QB_CHECK(stream, QBSM_ERR_ARG, "graph capture needs a non-null stream");
        Batch &b = batch->b;
        hipStream_t s = as_stream(stream);
        batch_settle(b, s);  // outside any capture
        if (!b.exec) {
            QB_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                batch_launch(b, s);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(s, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            QB_HIP(hipStreamEndCapture(s, &b.graph));
            QB_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
        }
        QB_HIP(hipGraphLaunch(b.exec, s));
    });
}

qbsm_status qbsm_batch_destroy(qbsm_batch batch) {
    return guard([&] {
        if (!batch) return;
        if (batch->b.exec) (void)hipGraphExecDestroy(batch->b.exec);
        if (batch->b.graph) (void)hipGraphDestroy(batch->b.graph);
        delete batch;
    });
}

qbsm_status qbsm_autotune_unit(qbsm_matrix A, qbsm_matrix B, qbsm_mode mode, int32_t reps, void *stream,
                               int32_t *best_unit, double *times_ms) {
    return guard([&] {
        QB_CHECK(A && B && best_unit, QBSM_ERR_ARG, "null argument");
        QB_CHECK(valid_mode(mode), QBSM_ERR_ARG, "unknown mode");
        QB_CHECK(reps >= 1, QBSM_ERR_ARG, "reps must be >= 1");
        hipStream_t s = as_stream(stream);
        const int bs = A->m.bs;
        const int cand[3] = {64, 128, 256};
        double best = -1.0;
        int bu = 0;
        hipEvent_t e0, e1;
        QB_HIP(hipEventCreate(&e0));
        QB_HIP(hipEventCreate(&e1));
        for (int ci = 0; ci < 3; ++ci) {
            const int u = cand[ci];
            double t = -1.0;
            const bool ok = (u % bs == 0) && (u / bs) <= 4 && (u / bs) >= 1 && !(u == 256 && mode == QBSM_F64) &&
                            !(mode == QBSM_OZAKI_I8 && ((u != 64 && u != 128) || bs != 64));
            if (ok) {
                auto p = plan_build(&A->m, 0, &B->m, 0, nullptr, u, 0.0, 0, s);
                Matrix out;
                out.nrows = p->out_rows;
                out.ncols = p->out_cols;
                out.bs = bs;
                out.nbr = (out.nrows + bs - 1) / bs;
                out.nbc = (out.ncols + bs - 1) / bs;
                numeric_prepare_output(*p, mode, out, s);
                numeric_launch(*p, mode, out, s);  // warm-up (packs operands)
                QB_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < reps; ++r) numeric_launch(*p, mode, out, s);
                QB_HIP(hipEventRecord(e1, s));
                QB_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                QB_HIP(hipEventElapsedTime(&ms, e0, e1));
                t = ms / reps;
                if (best < 0 || t < best) {
                    best = t;
                    bu = u;
                }
            }
            if (times_ms) times_ms[ci] = t;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *best_unit = bu;
    });
}

qbsm_status qbsm_batch_autotune(int32_t n, const qbsm_matrix *L, const qbsm_matrix *R, qbsm_mode mode, int32_t reps,
                                void *stream, qbsm_batch_tuning *out) {
    return guard([&] {
        QB_CHECK(n >= 1 && L && R && out, QBSM_ERR_ARG, "null argument or empty member list");
        QB_CHECK(valid_mode(mode), QBSM_ERR_ARG, "unknown mode");
        QB_CHECK(reps >= 1, QBSM_ERR_ARG, "reps must be >= 1");
        for (int i = 0; i < n; ++i) QB_CHECK(L[i] && R[i], QBSM_ERR_ARG, "null member matrix");
        hipStream_t s = as_stream(stream);
        qbsm_batch_tuning res{};
        for (auto &row : res.times_ms)
            for (double &t : row) t = -1.0;
        res.ms = -1.0;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        QB_HIP(hipEventCreate(&e0));
        QB_HIP(hipEventCreate(&e1));
        struct Events {
            hipEvent_t a, b;
            ~Events() {
                if (a) (void)hipEventDestroy(a);
                if (b) (void)hipEventDestroy(b);
            }
        } ev{e0, e1};
        const int cand[3] = {64, 128, 256};
        for (int ci = 0; ci < 3; ++ci) {
            const int u = cand[ci];
            bool ok = !(u == 256 && mode == QBSM_F64);
            for (int i = 0; i < n && ok; ++i) {
                const int bs = L[i]->m.bs;
                ok = u % bs == 0 && u / bs <= 4 && !(mode == QBSM_OZAKI_I8 && ((u != 64 && u != 128) || bs != 64));
            }
            if (!ok) continue;
            std::vector<std::unique_ptr<Plan>> plans;
            std::vector<std::unique_ptr<Matrix>> outs;
            std::vector<Plan *> pp;
            std::vector<Matrix *> op;
            for (int i = 0; i < n; ++i) {
                plans.push_back(plan_build(&L[i]->m, 0, &R[i]->m, 0, nullptr, u, 0.0, 0, s));
                auto o = std::make_unique<Matrix>();
                o->nrows = plans.back()->out_rows;
                o->ncols = plans.back()->out_cols;
                o->bs = L[i]->m.bs;
                o->nbr = (o->nrows + o->bs - 1) / o->bs;
                o->nbc = (o->ncols + o->bs - 1) / o->bs;
                pp.push_back(plans.back().get());
                op.push_back(o.get());
                outs.push_back(std::move(o));
            }
            Batch b;  // destroyed before the plans and outputs it points to
            batch_init(b, pp, op, mode, s);
            const int maxocc = std::min(4, k5_occupancy(mode, u, 0));
            for (int occ = 1; occ <= maxocc; ++occ) {
                b.wg_per_cu = occ;
                batch_settle(b, s);
                batch_launch(b, s);  // warm-up (packs, caches)
                QB_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < reps; ++r) batch_launch(b, s);
                QB_HIP(hipEventRecord(e1, s));
                QB_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                QB_HIP(hipEventElapsedTime(&ms, e0, e1));
                const double t = (double)ms / reps;
                res.times_ms[ci][occ - 1] = t;
                if (res.ms < 0 || t < res.ms) {
                    res.ms = t;
                    res.unit = u;
                    res.wg_per_cu = occ;
                }
            }
            QB_HIP(hipStreamSynchronize(s));
        }
        QB_CHECK(res.unit != 0, QBSM_ERR_UNSUPPORTED, "no unit side serves every member in this mode");
        *out = res;
    });
}

qbsm_status qbsm_profile_enable(int32_t on) {
    return guard([&] { g_prof.on = on != 0; });
}

qbsm_status qbsm_profile_reset(void) {
    return guard([&] {
        for (auto &v : g_prof.ev) {
            for (auto &p : v) {
                QB_HIP(hipEventSynchronize(p.second));
                g_prof.pool.push_back(p.first);
                g_prof.pool.push_back(p.second);
            }
            v.clear();
        }
    });
}

qbsm_status qbsm_profile_read(int32_t kernel_class, int64_t *launches, double *total_ms) {
    return guard([&] {
        QB_CHECK(kernel_class >= 0 && kernel_class < PROF_NCLASS, QBSM_ERR_ARG, "kernel class");
        double tot = 0.0;
        for (auto &p : g_prof.ev[kernel_class]) {
            QB_HIP(hipEventSynchronize(p.second));
            float ms = 0.f;
            QB_HIP(hipEventElapsedTime(&ms, p.first, p.second));
            tot += ms;
        }
        if (launches) *launches = (int64_t)g_prof.ev[kernel_class].size();
        if (total_ms) *total_ms = tot;
    });
}

}  // extern "C"
