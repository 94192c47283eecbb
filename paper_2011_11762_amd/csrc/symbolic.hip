// Symbolic phase: level-synchronous walk of two sparse quadtrees.
//
// The paper's multiply task (Sec. 2 and 2.1) handles one quadtree level per
// task: for a non-leaf output quadrant C_ij it registers the child products
// A_ik * B_kj, k in {0,1}, and any product with a nil operand is skipped
// (the nil fallback).  Here all tasks of one level are expanded at once.  A
// "pair" is a live product (L node at (i,k), R node at (k,j)) of one level;
// pairs are kept grouped by output node (Morton order) and, inside a group,
// ordered by the contraction index k.  Expanding a group quadrant by
// quadrant and, inside a quadrant, pair by pair with the child index kb
// ascending keeps both orders at the next level, so no sort is needed: at
// the leaves every output block's products come out contiguous with K
// ascending.
#include "common.h"

namespace qbsm {

namespace {

struct Pairs {
    int64_t n = 0;
    DArr<int32_t> pl, pr, gs, gm, pm;
    DArr<uint32_t> ck;
    void alloc(int64_t cnt, hipStream_t s) {
        const int64_t c = cnt ? cnt : 1;
        n = cnt;
        pl.alloc(c, s); pr.alloc(c, s); gs.alloc(c, s); gm.alloc(c, s); pm.alloc(c, s); ck.alloc(c, s);
    }
};

__device__ __forceinline__ int slot_of(int rowbit, int colbit, int trans) {
    return trans ? (colbit * 2 + rowbit) : (rowbit * 2 + colbit);
}

__global__ void k_walk_count(int64_t np, const int32_t *pl, const int32_t *pr, const int32_t *gs,
                             const int32_t *gm, const int32_t *pm, const int32_t *chL, const int32_t *chR,
                             const int32_t *chM, int transL, int transR, int32_t *X) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np * 4) return;
    const int64_t p = t >> 2;
    const int q = (int)(t & 3);
    const int ib = q >> 1, jb = q & 1;
    int cnt = 0;
    if (!chM || chM[(int64_t)pm[p] * 4 + q] >= 0) {
        const int64_t a = (int64_t)pl[p] * 4, b = (int64_t)pr[p] * 4;
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const int32_t cl = chL[a + slot_of(ib, kb, transL)];
            const int32_t cr = chR[b + slot_of(kb, jb, transR)];
            cnt += (cl >= 0 && cr >= 0) ? 1 : 0;
        }
    }
    const int64_t g = gs[p];
    X[4 * g + (int64_t)q * gm[p] + (p - g)] = cnt;
}

__global__ void k_walk_fill(int64_t np, const int32_t *pl, const int32_t *pr, const int32_t *gs,
                            const int32_t *gm, const int32_t *pm, const uint32_t *ck, const int32_t *chL,
                            const int32_t *chR, const int32_t *chM, int transL, int transR,
                            const int32_t *Y, int32_t *opl, int32_t *opr, int32_t *ogs, int32_t *ogm,
                            int32_t *opm, uint32_t *ock) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np * 4) return;
    const int64_t p = t >> 2;
    const int q = (int)(t & 3);
    const int ib = q >> 1, jb = q & 1;
    int32_t mchild = -1;
    if (chM) {
        mchild = chM[(int64_t)pm[p] * 4 + q];
        if (mchild < 0) return;
    }
    const int64_t g = gs[p], m = gm[p];
    const int64_t base = 4 * g + (int64_t)q * m;
    int32_t o = Y[base + (p - g)];
    const int32_t ngs = Y[base];
    const int32_t nge = Y[base + m];
    const int64_t a = (int64_t)pl[p] * 4, b = (int64_t)pr[p] * 4;
    const uint32_t key = ck[p] * 4u + (uint32_t)q;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        const int32_t cl = chL[a + slot_of(ib, kb, transL)];
        const int32_t cr = chR[b + slot_of(kb, jb, transR)];
        if (cl >= 0 && cr >= 0) {
            opl[o] = cl;
            opr[o] = cr;
            ogs[o] = ngs;
            ogm[o] = nge - ngs;
            opm[o] = mchild;
            ock[o] = key;
            ++o;
        }
    }
}

__global__ void k_walk_root(int32_t *pl, int32_t *pr, int32_t *gs, int32_t *gm, int32_t *pm, uint32_t *ck) {
    pl[0] = 0; pr[0] = 0; gs[0] = 0; gm[0] = 1; pm[0] = 0; ck[0] = 0u;
}

// Runs the walk from the root to level `target`; returns the pair list there.
Pairs walk(Tree &tL, int transL, Tree &tR, int transR, Tree *tM, int target, hipStream_t s) {
    Pairs cur;
    const bool empty = tL.n[0] == 0 || tR.n[0] == 0 || (tM && tM->n[0] == 0);
    cur.alloc(empty ? 0 : 1, s);
    if (!empty) {
        k_walk_root<<<1, 1, 0, s>>>(cur.pl.p, cur.pr.p, cur.gs.p, cur.gm.p, cur.pm.p, cur.ck.p);
        QB_LAUNCH_CHECK();
    }
    DArr<int64_t> tot(1, s);
    for (int l = 0; l < target && cur.n > 0; ++l) {
        const int64_t np = cur.n;
        DArr<int32_t> X(np * 4, s), Y(np * 4 + 1, s);
        const unsigned g = grid_for(np * 4, 256);
        const int32_t *chM = tM ? tM->child[l].p : nullptr;
        k_walk_count<<<g, 256, 0, s>>>(np, cur.pl.p, cur.pr.p, cur.gs.p, cur.gm.p, cur.pm.p, tL.child[l].p,
                                      tR.child[l].p, chM, transL, transR, X.p);
        QB_LAUNCH_CHECK();
        exclusive_scan_i32(X.p, Y.p, np * 4, tot.p, s);
        const int64_t nn = read_back(tot.p, s);
        QB_CHECK(nn <= (int64_t)INT32_MAX, QBSM_ERR_UNSUPPORTED, "too many node pairs at one level");
        Pairs nxt;
        nxt.alloc(nn, s);
        if (nn) {
            k_walk_fill<<<g, 256, 0, s>>>(np, cur.pl.p, cur.pr.p, cur.gs.p, cur.gm.p, cur.pm.p, cur.ck.p,
                                         tL.child[l].p, tR.child[l].p, chM, transL, transR, Y.p, nxt.pl.p,
                                         nxt.pr.p, nxt.gs.p, nxt.gm.p, nxt.pm.p, nxt.ck.p);
            QB_LAUNCH_CHECK();
        }
        cur = std::move(nxt);
    }
    return cur;
}

__device__ __forceinline__ int morton_sub(int r, int c, int s) {
    // interleave the s low bits of r and c, r's bit above c's
    int q = 0;
    for (int b = 0; b < s; ++b) q |= (((r >> b) & 1) << (2 * b + 1)) | (((c >> b) & 1) << (2 * b));
    return q;
}

__device__ __forceinline__ void demorton_u32(uint32_t k, uint32_t &i, uint32_t &j) {
    i = 0;
    j = 0;
    for (int b = 0; b < 16; ++b) {
        i |= ((k >> (2 * b + 1)) & 1u) << b;
        j |= ((k >> (2 * b)) & 1u) << b;
    }
}

__global__ void k_unit_flags(int64_t np, const int32_t *gs, int32_t *flags) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < np) flags[p] = (gs[p] == (int32_t)p) ? 1 : 0;
}

__global__ void k_unit_fill(int64_t np, const int32_t *gs, const int32_t *pm, const uint32_t *ck,
                            const int32_t *uscan, int32_t *ustart, uint32_t *ukey, int32_t *umask,
                            int32_t *pu) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const bool start = gs[p] == (int32_t)p;
    const int32_t u = uscan[p] + (start ? 1 : 0) - 1;
    pu[p] = u;
    if (start) {
        ustart[u] = (int32_t)p;
        ukey[u] = ck[p];
        umask[u] = pm[p];
    }
}

__global__ void k_unit_end(int32_t *ustart, int64_t nunits, int64_t np) { ustart[nunits] = (int32_t)np; }

struct Dims {
    int64_t out_rows, inner, out_cols;
    int32_t bs, s, lpu, transL, transR;
};

__device__ __forceinline__ int64_t ext(int64_t idx, int64_t n, int32_t bs) {
    const int64_t e = n - idx * bs;
    return e < bs ? e : bs;
}

// Leaf-product bits of each unit-level pair, output-leaf bits of each unit,
// product and flop totals.
__global__ void k_pair_masks(int64_t np, const int32_t *pl, const int32_t *pr, const int32_t *pu,
                             const uint32_t *ukey, const int32_t *umask, const int32_t *descL,
                             const int32_t *descR, const int32_t *descM, int hasM, const uint32_t *keyL,
                             Dims d, uint64_t *pmask, uint32_t *ucmask, unsigned long long *nprod,
                             unsigned long long *flops) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int lpu = d.lpu, s = d.s, nsub = lpu * lpu;
    const int32_t a = pl[p], b = pr[p];
    const int32_t u = pu[p];
    uint32_t ui, uj, lr, lc;
    demorton_u32(ukey[u], ui, uj);
    demorton_u32(keyL[a], lr, lc);
    const uint32_t uk = d.transL ? lr : lc;  // contraction coordinate of the L node
    uint64_t bits = 0;
    uint32_t cm = 0;
    unsigned long long fl = 0;
    for (int kb = 0; kb < lpu; ++kb) {
        for (int ib = 0; ib < lpu; ++ib) {
            const int qa = d.transL ? morton_sub(kb, ib, s) : morton_sub(ib, kb, s);
            const int32_t la = descL ? descL[(int64_t)a * nsub + qa] : a;
            if (la < 0) continue;
            for (int jb = 0; jb < lpu; ++jb) {
                const int qb = d.transR ? morton_sub(jb, kb, s) : morton_sub(kb, jb, s);
                const int32_t lb = descR ? descR[(int64_t)b * nsub + qb] : b;
                if (lb < 0) continue;
                if (hasM) {
                    const int32_t lm = descM ? descM[(int64_t)umask[u] * nsub + morton_sub(ib, jb, s)] : umask[u];
                    if (lm < 0) continue;
                }
                bits |= 1ull << ((kb * lpu + ib) * lpu + jb);
                cm |= 1u << (ib * lpu + jb);
                const int64_t I = (int64_t)ui * lpu + ib, J = (int64_t)uj * lpu + jb, K = (int64_t)uk * lpu + kb;
                fl += (unsigned long long)(2 * ext(I, d.out_rows, d.bs) * ext(K, d.inner, d.bs) *
                                           ext(J, d.out_cols, d.bs));
            }
        }
    }
    pmask[p] = bits;
    if (cm) atomicOr(&ucmask[u], cm);
    const int np_ = __popcll(bits);
    if (np_) {
        atomicAdd(nprod, (unsigned long long)np_);
        atomicAdd(flops, fl);
    }
}

__global__ void k_unit_count(int64_t nu, const uint32_t *ucmask, int32_t *cnt) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < nu) cnt[u] = __popc(ucmask[u]);
}

// Output leaves of each unit: numbered in Morton order inside the unit
// (unmasked plans), or taken from the mask's leaves (masked plans).
__global__ void k_unit_cdesc(int64_t nu, const uint32_t *ucmask, const int32_t *cbase, const uint32_t *ukey,
                             const int32_t *umask, const int32_t *descM, int hasM, int s, int lpu,
                             int32_t *cdesc, uint32_t *okeys) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nu) return;
    const uint32_t cm = ucmask[u];
    const int nsub = lpu * lpu;
    int32_t next = hasM ? 0 : cbase[u];
    for (int q = 0; q < nsub; ++q) {
        // q is the Morton sub-index; recover (ib, jb)
        int ib = 0, jb = 0;
        for (int b = 0; b < s; ++b) {
            ib |= ((q >> (2 * b + 1)) & 1) << b;
            jb |= ((q >> (2 * b)) & 1) << b;
        }
        const int rm = ib * lpu + jb;
        int32_t v = -1;
        if ((cm >> rm) & 1u) {
            if (hasM) {
                v = descM ? descM[(int64_t)umask[u] * nsub + q] : umask[u];
            } else {
                v = next++;
                okeys[v] = (ukey[u] << (2 * s)) | (uint32_t)q;
            }
        }
        cdesc[u * nsub + rm] = v;
    }
}

// ---- product export (canonical row-major output, K ascending)
__global__ void k_leaf_groups(int64_t np, const int32_t *gs, const uint32_t *ck, int64_t nbc, int32_t *gflag,
                              uint32_t *rmk) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const bool start = gs[p] == (int32_t)p;
    gflag[p] = start ? 1 : 0;
    if (start) {
        uint32_t i, j;
        demorton_u32(ck[p], i, j);
        rmk[p] = (uint32_t)((uint64_t)i * nbc + j);
    }
}

__global__ void k_i32_to_u8(const int32_t *f, uint8_t *a, int64_t n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = (uint8_t)f[t];
}

__global__ void k_group_sizes(int64_t np, const int32_t *gs, const int32_t *gm, const int32_t *grank,
                              int32_t *size_by_rank) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    if (gs[p] == (int32_t)p) size_by_rank[grank[p]] = gm[p];
}

__global__ void k_emit_products(int64_t np, const int32_t *gs, const int32_t *pl, const uint32_t *ck,
                                const int32_t *grank, const int32_t *off, const uint32_t *keyL, int transL,
                                int32_t *I, int32_t *K, int32_t *J) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int32_t g = gs[p];
    const int32_t pos = off[grank[g]] + (int32_t)(p - g);
    uint32_t i, j, r, c;
    demorton_u32(ck[p], i, j);
    demorton_u32(keyL[pl[p]], r, c);
    I[pos] = (int32_t)i;
    J[pos] = (int32_t)j;
    K[pos] = (int32_t)(transL ? r : c);
}

}  // namespace

std::unique_ptr<Plan> plan_build(Matrix *L, int transL, Matrix *R, int transR, Matrix *M, int unit,
                                 hipStream_t s) {
    QB_CHECK(L && R, QBSM_ERR_ARG, "null matrix");
    QB_CHECK(L->has_blocks && R->has_blocks && (!M || M->has_blocks), QBSM_ERR_STATE,
             "matrix has no blocks yet");
    QB_CHECK(L->bs == R->bs && (!M || M->bs == L->bs), QBSM_ERR_SHAPE, "leaf sizes differ");
    const int bs = L->bs;
    const int64_t rows = transL ? L->ncols : L->nrows;
    const int64_t inner = transL ? L->nrows : L->ncols;
    const int64_t innerR = transR ? R->ncols : R->nrows;
    const int64_t cols = transR ? R->nrows : R->ncols;
    QB_CHECK(inner == innerR, QBSM_ERR_SHAPE, "inner dimensions differ");
    if (M) QB_CHECK(M->nrows == rows && M->ncols == cols, QBSM_ERR_SHAPE, "mask shape differs from the product");
    if (unit == 0) unit = 128;
    int sl = -1;
    for (int t = 0; t <= 2; ++t)
        if ((bs << t) == unit) sl = t;
    QB_CHECK(sl >= 0 && (unit == 64 || unit == 128 || unit == 256), QBSM_ERR_UNSUPPORTED,
             "unit must be bs*2^s (s<=2) and one of 64, 128, 256");
    const int64_t nbI = (rows + bs - 1) / bs, nbK = (inner + bs - 1) / bs, nbJ = (cols + bs - 1) / bs;
    int64_t nbmax = nbI > nbK ? nbI : nbK;
    nbmax = nbmax > nbJ ? nbmax : nbJ;
    int D = ceil_log2(nbmax < 1 ? 1 : nbmax);
    if (D < sl) D = sl;
    QB_CHECK(D <= 16, QBSM_ERR_UNSUPPORTED, "block grid side above 65536");

    static uint64_t next_id = 0;
    auto p = std::make_unique<Plan>();
    p->id = ++next_id;
    p->L = L; p->R = R; p->M = M;
    p->transL = transL; p->transR = transR;
    p->patL = L->pattern_id; p->patR = R->pattern_id; p->patM = M ? M->pattern_id : 0;
    p->D = D; p->s = sl; p->unit = unit; p->bs = bs; p->lpu = 1 << sl;
    p->out_rows = rows; p->out_cols = cols;
    p->stream = s;

    Tree &tL = matrix_tree(*L, D, s);
    Tree &tR = matrix_tree(*R, D, s);
    Tree *tM = M ? &matrix_tree(*M, D, s) : nullptr;
    const int Lw = D - sl;
    Pairs pr = walk(tL, transL, tR, transR, tM, Lw, s);
    const int64_t np = pr.n;
    p->npairs = np;
    const int nsub = p->lpu * p->lpu;

    // units = output groups at the unit level
    DArr<int32_t> flags(np ? np : 1, s), uscan((np ? np : 1) + 1, s), pu(np ? np : 1, s);
    DArr<int64_t> tot(1, s);
    int64_t nu = 0;
    if (np) {
        k_unit_flags<<<grid_for(np, 256), 256, 0, s>>>(np, pr.gs.p, flags.p);
        QB_LAUNCH_CHECK();
        exclusive_scan_i32(flags.p, uscan.p, np, tot.p, s);
        nu = read_back(tot.p, s);
    }
    p->nunits = nu;
    p->ustart.alloc(nu + 1, s);
    p->ukey.alloc(nu ? nu : 1, s);
    p->umask.alloc(nu ? nu : 1, s);
    p->pl = std::move(pr.pl);
    p->pr = std::move(pr.pr);
    p->pmask.alloc(np ? np : 1, s);
    p->cdesc.alloc((nu ? nu : 1) * nsub, s);
    struct Tot { unsigned long long nprod, flops; };
    DArr<Tot> totals(1, s);
    QB_HIP(hipMemsetAsync(totals.p, 0, sizeof(Tot), s));
    DArr<uint32_t> ucmask(nu ? nu : 1, s);
    fill_u32(ucmask.p, 0u, nu ? nu : 1, s);
    if (np) {
        k_unit_fill<<<grid_for(np, 256), 256, 0, s>>>(np, pr.gs.p, pr.pm.p, pr.ck.p, uscan.p, p->ustart.p,
                                                     p->ukey.p, p->umask.p, pu.p);
        QB_LAUNCH_CHECK();
        k_unit_end<<<1, 1, 0, s>>>(p->ustart.p, nu, np);
        QB_LAUNCH_CHECK();
        Dims d{rows, inner, cols, bs, sl, p->lpu, transL, transR};
        const int32_t *dL = tree_desc(*L, tL, sl, s);
        const int32_t *dR = tree_desc(*R, tR, sl, s);
        const int32_t *dM = M ? tree_desc(*M, *tM, sl, s) : nullptr;
        k_pair_masks<<<grid_for(np, 256), 256, 0, s>>>(np, p->pl.p, p->pr.p, pu.p, p->ukey.p, p->umask.p, dL,
                                                      dR, dM, M ? 1 : 0, tL.key[Lw].p, d, p->pmask.p,
                                                      ucmask.p, &totals.p->nprod, &totals.p->flops);
        QB_LAUNCH_CHECK();
    } else {
        int32_t zero = 0;
        QB_HIP(hipMemcpyAsync(p->ustart.p, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    // output leaves
    int64_t nout = 0;
    if (nu) {
        DArr<int32_t> cnt(nu, s), cbase(nu + 1, s);
        k_unit_count<<<grid_for(nu, 256), 256, 0, s>>>(nu, ucmask.p, cnt.p);
        QB_LAUNCH_CHECK();
        exclusive_scan_i32(cnt.p, cbase.p, nu, tot.p, s);
        nout = read_back(tot.p, s);
        if (!M) p->okeys.alloc(nout ? nout : 1, s);
        const int32_t *dM = M ? tree_desc(*M, *tM, sl, s) : nullptr;
        k_unit_cdesc<<<grid_for(nu, 256), 256, 0, s>>>(nu, ucmask.p, cbase.p, p->ukey.p, p->umask.p, dM,
                                                      M ? 1 : 0, sl, p->lpu, p->cdesc.p,
                                                      M ? nullptr : p->okeys.p);
        QB_LAUNCH_CHECK();
    } else if (!M) {
        p->okeys.alloc(1, s);
    }
    Tot h = read_back(totals.p, s);
    p->nprod = (int64_t)h.nprod;
    p->flops = (int64_t)h.flops;
    p->nout = M ? M->nblk : nout;
    return p;
}

void plan_get_products(Plan &p, int32_t *I, int32_t *K, int32_t *J, hipStream_t s) {
    if (!p.nprod) return;
    Tree &tL = matrix_tree(*p.L, p.D, s);
    Tree &tR = matrix_tree(*p.R, p.D, s);
    Tree *tM = p.M ? &matrix_tree(*p.M, p.D, s) : nullptr;
    Pairs lv = walk(tL, p.transL, tR, p.transR, tM, p.D, s);
    const int64_t np = lv.n;
    QB_CHECK(np == p.nprod, QBSM_ERR_STATE, "leaf walk disagrees with the plan's product count");
    const int64_t nbc = (p.out_cols + p.bs - 1) / p.bs;
    const int64_t nbr = (p.out_rows + p.bs - 1) / p.bs;
    DArr<int32_t> gflag(np, s), grank(np, s), sizes(np, s), off(np + 1, s), dup(1, s);
    DArr<uint32_t> rmk(np, s);
    DArr<int64_t> cnt(1, s);
    k_leaf_groups<<<grid_for(np, 256), 256, 0, s>>>(np, lv.gs.p, lv.ck.p, nbc, gflag.p, rmk.p);
    QB_LAUNCH_CHECK();
    // rank the groups (output blocks) in row-major order; gflag marks starts
    DArr<uint8_t> act(np, s);
    k_i32_to_u8<<<grid_for(np, 256), 256, 0, s>>>(gflag.p, act.p, np);
    QB_LAUNCH_CHECK();
    bitmap_rank(rmk.p, act.p, np, (uint64_t)nbr * (uint64_t)nbc, grank.p, dup.p, cnt.p, s);
    fill_i32(sizes.p, 0, np, s);
    k_group_sizes<<<grid_for(np, 256), 256, 0, s>>>(np, lv.gs.p, lv.gm.p, grank.p, sizes.p);
    QB_LAUNCH_CHECK();
    exclusive_scan_i32(sizes.p, off.p, np, cnt.p, s);
    k_emit_products<<<grid_for(np, 256), 256, 0, s>>>(np, lv.gs.p, lv.pl.p, lv.ck.p, grank.p, off.p,
                                                     tL.key[p.D].p, p.transL, I, K, J);
    QB_LAUNCH_CHECK();
}

}  // namespace qbsm
