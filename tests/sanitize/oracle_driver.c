/*
 * Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * CPU oracle's C part (test infrastructure).  Runs both entry points on small
 * inputs with edge cases (no output blocks, empty segments, every transpose
 * combination, leaf size 1) and checks them against naive loops in the same
 * summation order, so equality is exact.  Exit status 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_block_fnorm(int64_t nblk, int32_t bs, const double *vals, double *out);
void oracle_segmented_products(int32_t bs, int64_t nout, const int64_t *seg, const int64_t *lidx,
                               const int64_t *ridx, const double *L, const double *R, int transL,
                               int transR, double *out);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double draw(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static double at(const double *x, int bs, int trans, int r, int c)
{
    return trans ? x[c + (int64_t)r * bs] : x[r + (int64_t)c * bs];
}

static int check_products(int bs, int nleaf, int nout, int maxseg, int tl, int tr)
{
    const int64_t n2 = (int64_t)bs * bs;
    double *L = malloc(sizeof(double) * (size_t)(nleaf * n2 + 1));
    double *R = malloc(sizeof(double) * (size_t)(nleaf * n2 + 1));
    int64_t *seg = malloc(sizeof(int64_t) * (size_t)(nout + 1));
    int64_t *li = malloc(sizeof(int64_t) * (size_t)(nout * maxseg + 1));
    int64_t *ri = malloc(sizeof(int64_t) * (size_t)(nout * maxseg + 1));
    double *out = malloc(sizeof(double) * (size_t)(nout * n2 + 1));
    double *ref = malloc(sizeof(double) * (size_t)(nout * n2 + 1));
    for (int64_t e = 0; e < nleaf * n2; ++e) {
        L[e] = draw();
        R[e] = draw();
    }
    seg[0] = 0;
    for (int o = 0; o < nout; ++o) {
        const int len = (int)((draw() + 1.0) * 0.5 * (maxseg + 1)) % (maxseg + 1);  /* 0 .. maxseg */
        for (int t = 0; t < len; ++t) {
            li[seg[o] + t] = (int64_t)((draw() + 1.0) * 0.5 * nleaf) % nleaf;
            ri[seg[o] + t] = (int64_t)((draw() + 1.0) * 0.5 * nleaf) % nleaf;
        }
        seg[o + 1] = seg[o] + len;
    }
    oracle_segmented_products(bs, nout, seg, li, ri, L, R, tl, tr, out);
    int bad = 0;
    for (int o = 0; o < nout; ++o) {
        double *c = ref + o * n2;
        for (int64_t e = 0; e < n2; ++e) c[e] = 0.0;
        for (int64_t t = seg[o]; t < seg[o + 1]; ++t)
            for (int j = 0; j < bs; ++j)
                for (int l = 0; l < bs; ++l)
                    for (int i = 0; i < bs; ++i)
                        c[i + (int64_t)j * bs] += at(L + li[t] * n2, bs, tl, i, l) * at(R + ri[t] * n2, bs, tr, l, j);
        for (int64_t e = 0; e < n2; ++e) bad |= c[e] != out[o * n2 + e];
    }
    free(L); free(R); free(seg); free(li); free(ri); free(out); free(ref);
    return bad;
}

int main(void)
{
    int bad = 0;
    /* norms, including an empty call */
    const int bs = 5;
    double v[3 * 25], nrm[3];
    for (int e = 0; e < 75; ++e) v[e] = draw();
    oracle_block_fnorm(0, bs, v, nrm);
    oracle_block_fnorm(3, bs, v, nrm);
    for (int b = 0; b < 3; ++b) {
        double s = 0.0;
        for (int e = 0; e < 25; ++e) s += v[b * 25 + e] * v[b * 25 + e];
        bad |= sqrt(s) != nrm[b];
    }
    /* products: no output blocks, leaf size 1, odd sizes, every transpose pair */
    bad |= check_products(4, 3, 0, 2, 0, 0);
    bad |= check_products(1, 4, 9, 3, 0, 0);
    for (int tl = 0; tl < 2; ++tl)
        for (int tr = 0; tr < 2; ++tr) {
            bad |= check_products(7, 6, 11, 4, tl, tr);
            bad |= check_products(16, 5, 7, 5, tl, tr);
        }
    if (bad) {
        fprintf(stderr, "oracle driver: results differ from the naive loops\n");
        return 1;
    }
    printf("oracle driver ok\n");
    return 0;
}
