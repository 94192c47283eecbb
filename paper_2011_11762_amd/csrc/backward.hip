// Masked backward from the forward product list.
//
// For C = A B the adjoints restricted to the operand patterns are
//   dA = (dC B^T) on A's pattern:  dA_IK = sum_J dC_IJ B_KJ^T,
//   dB = (A^T dC) on B's pattern:  dB_KJ = sum_I A_IK^T dC_IJ,
// and every term is one forward leaf product (I, K, J) whose dC block exists.
// So the backward needs no symbolic walk: the forward plan's unit-level
// pairs (A node (i,k), B node (k,j)) of output unit (i,j) are regrouped by
// their A node (for dA; each becomes the pair (dC node (i,j), B node (k,j)),
// contraction over j) or by their B node (for dB; the pair (A node (i,k),
// dC node (i,j)), contraction over i), and each pair's leaf-product bits are
// re-indexed and cut to the dC leaves that exist.  A stable radix sort on
// the new output node keeps the forward order inside every group, so the
// summation order is fixed and repeated runs are bit-identical.  The result
// is a masked plan on the regular numeric kernel; mask blocks without
// products come out zero.
#include <hipcub/hipcub.hpp>

#include "common.h"
#include "trees.h"

namespace qbsm {

namespace {

__device__ __forceinline__ int msub_dyn(int r, int c, int s) {
    int q = 0;
    for (int b = 0; b < s; ++b) q |= (((r >> b) & 1) << (2 * b + 1)) | (((c >> b) & 1) << (2 * b));
    return q;
}

// Sort keys: the forward pair's A node (dA) or B node (dB).
__global__ void k_bwd_keys(int64_t np, const int32_t *node, uint32_t *key, int32_t *idx) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    key[p] = (uint32_t)node[p];
    idx[p] = (int32_t)p;
}

// First sorted position of every output node (ustart), by binary search.
__global__ void k_bwd_ustart(int64_t nout, int64_t np, const uint32_t *skey, int32_t *ustart) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > nout) return;
    int64_t lo = 0, hi = np;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)skey[mid] < u) lo = mid + 1; else hi = mid;
    }
    ustart[u] = (int32_t)lo;
}

// Index of `key` among the n ascending keys, -1 if absent.
__device__ __forceinline__ int32_t find_key(const uint32_t *keys, int64_t n, uint32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && keys[lo] == key) ? (int32_t)lo : -1;
}

// One regrouped pair per sorted position.  which 0: dA (L = dC, R = B
// transposed); which 1: dB (L = A transposed, R = dC).  The forward bit
// ((kb*LPU + ib)*LPU + jb) is the leaf product A(ib,kb) B(kb,jb) of the
// pair's output unit (i,j); dC's sub-leaf (ib,jb) must exist.
__global__ void k_bwd_pairs(int64_t np, int which, int s, const int32_t *sidx, const int32_t *fstart,
                            int64_t fnunits, const uint32_t *fukey, const int32_t *fpl, const int32_t *fpr,
                            const uint64_t *fpmask, const uint32_t *dckeys, int64_t ndc, const int32_t *dcdesc,
                            int32_t *pl, int32_t *pr, uint64_t *pmask) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    const int32_t p = sidx[q];
    // forward unit of pair p: the last unit starting at or before p
    int64_t lo = 0, hi = fnunits;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (fstart[mid] <= p) lo = mid; else hi = mid;
    }
    const int32_t dcn = find_key(dckeys, ndc, fukey[lo]);
    const int lpu = 1 << s, nsub = lpu * lpu;
    const uint64_t fb = fpmask[p];
    uint64_t bits = 0;
    if (dcn >= 0) {
        for (int kb = 0; kb < lpu; ++kb)
            for (int ib = 0; ib < lpu; ++ib)
                for (int jb = 0; jb < lpu; ++jb) {
                    if (!((fb >> ((kb * lpu + ib) * lpu + jb)) & 1ull)) continue;
                    const bool dc = s == 0 ? true : dcdesc[(int64_t)dcn * nsub + msub_dyn(ib, jb, s)] >= 0;
                    if (!dc) continue;
                    // dA: out (ib,kb), contraction jb; dB: out (kb,jb), contraction ib
                    const int bit = which == 0 ? (jb * lpu + ib) * lpu + kb : (ib * lpu + kb) * lpu + jb;
                    bits |= 1ull << bit;
                }
    }
    if (which == 0) {
        pl[q] = dcn >= 0 ? dcn : 0;  // a pair without products is skipped by the kernel
        pr[q] = fpr[p];
    } else {
        pl[q] = fpl[p];
        pr[q] = dcn >= 0 ? dcn : 0;
    }
    pmask[q] = bits;
}

// Output leaves of every unit (an operand node at the unit level): the
// operand's own leaves, so the result keeps its pattern.
__global__ void k_bwd_cdesc(int64_t nu, int s, const int32_t *desc, int32_t *cdesc, int32_t *umask) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nu) return;
    const int lpu = 1 << s, nsub = lpu * lpu;
    umask[u] = (int32_t)u;
    for (int ib = 0; ib < lpu; ++ib)
        for (int jb = 0; jb < lpu; ++jb)
            cdesc[u * nsub + ib * lpu + jb] = s == 0 ? (int32_t)u : desc[u * nsub + msub_dyn(ib, jb, s)];
}

}  // namespace

bool plan_backward_ok(const Plan &f) {
    return !f.transL && !f.transR && !f.M && f.spamm_tol <= 0.0 && !f.upper;
}

std::unique_ptr<Plan> plan_backward(const Plan &f, Matrix *dC, int which, hipStream_t s) {
    QB_CHECK(plan_backward_ok(f), QBSM_ERR_UNSUPPORTED,
             "the backward regroups a regular forward plan (no transposes, mask, approximation or triangle)");
    plan_check_current(f);
    QB_CHECK(dC && dC->has_blocks, QBSM_ERR_STATE, "dC has no blocks");
    QB_CHECK(dC->nrows == f.out_rows && dC->ncols == f.out_cols && dC->bs == f.bs, QBSM_ERR_SHAPE,
             "dC shape or leaf size differs from the product");
    Matrix *X = which == 0 ? f.L : f.R;  // the operand whose adjoint is formed (its pattern is the mask)
    const int Lw = f.D - f.s;
    Matrix *const ops[2] = {X, dC};
    matrix_trees(ops, 2, f.D, s);
    Tree &tX = matrix_tree(*X, f.D, s);
    Tree &tC = matrix_tree(*dC, f.D, s);
    static uint64_t next_id = 0;
    auto p = std::make_unique<Plan>();
    p->id = (uint64_t(1) << 62) | ++next_id;
    p->sched = f.sched;  // the forward plan's numeric schedule
    if (which == 0) {
        p->L = dC; p->transL = 0; p->R = f.R; p->transR = 1;
    } else {
        p->L = f.L; p->transL = 1; p->R = dC; p->transR = 0;
    }
    p->M = X;
    p->patL = p->L->pattern_id;
    p->patR = p->R->pattern_id;
    p->patM = X->pattern_id;
    p->D = f.D; p->s = f.s; p->unit = f.unit; p->bs = f.bs; p->lpu = f.lpu;
    p->out_rows = X->nrows;
    p->out_cols = X->ncols;
    p->stream = s;
    const int64_t np = f.npairs, nu = tX.n[Lw];
    const int nsub = f.lpu * f.lpu;
    p->npairs = np;
    p->nunits = np ? nu : 0;
    p->nout = X->nblk;
    p->ustart.alloc(p->nunits + 1, s);
    p->ukey.alloc(nu ? nu : 1, s);
    p->umask.alloc(nu ? nu : 1, s);
    p->pl.alloc(np ? np : 1, s);
    p->pr.alloc(np ? np : 1, s);
    p->pmask.alloc(np ? np : 1, s);
    p->cdesc.alloc((nu ? nu : 1) * nsub, s);
    if (!np) {
        fill_i32(p->ustart.p, 0, 1, s);
        return p;
    }
    // stable sort of the forward pairs by their node of X
    DArr<uint32_t> key(np, s), skey(np, s);
    DArr<int32_t> idx(np, s), sidx(np, s);
    k_bwd_keys<<<grid_for(np, 256), 256, 0, s>>>(np, which == 0 ? f.pl.p : f.pr.p, key.p, idx.p);
    QB_LAUNCH_CHECK();
    const int bits = ceil_log2(nu < 2 ? 2 : nu);
    size_t tmp_bytes = 0;
    QB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key.p, skey.p, idx.p, sidx.p, (int)np, 0, bits, s));
    DArr<uint8_t> tmp(tmp_bytes ? tmp_bytes : 1, s);
    QB_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, key.p, skey.p, idx.p, sidx.p, (int)np, 0, bits, s));
    k_bwd_ustart<<<grid_for(nu + 1, 256), 256, 0, s>>>(nu, np, skey.p, p->ustart.p);
    QB_LAUNCH_CHECK();
    const int32_t *dcdesc = tree_desc(*dC, tC, f.s, s);
    k_bwd_pairs<<<grid_for(np, 256), 256, 0, s>>>(np, which, f.s, sidx.p, f.ustart.p, f.nunits, f.ukey.p, f.pl.p,
                                                  f.pr.p, f.pmask.p, tC.key[Lw].p, tC.n[Lw], dcdesc, p->pl.p,
                                                  p->pr.p, p->pmask.p);
    QB_LAUNCH_CHECK();
    QB_HIP(hipMemcpyAsync(p->ukey.p, tX.key[Lw].p, nu * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    const int32_t *xdesc = tree_desc(*X, tX, f.s, s);
    k_bwd_cdesc<<<grid_for(nu, 256), 256, 0, s>>>(nu, f.s, xdesc, p->cdesc.p, p->umask.p);
    QB_LAUNCH_CHECK();
    // the other operand's tables at the plan's depth, for the numeric phase
    (void)tree_desc(*(which == 0 ? f.R : f.L), matrix_tree(*(which == 0 ? f.R : f.L), f.D, s), f.s, s);
    return p;
}

}  // namespace qbsm
