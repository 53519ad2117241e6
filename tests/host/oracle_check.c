/* A small run of the oracle's entry points (columns with hit lists, rates, a
 * solve, the reference trees, slab solutions) built with the address and
 * undefined-behaviour sanitizers by tests/test_host_sanitized.py. */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#define CHECK(cond)                                                            \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            exit(1);                                                           \
        }                                                                      \
    } while (0)

int main(void)
{
    enum { N = 64, NR = 6 };
    float pos[3 * N], h[N], mu[N], nH[N], T[N];
    double x[N], dirs[3 * NR] = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
    for (int i = 0; i < N; ++i) {
        pos[3 * i] = (float)(i % 4) * 2.5f + 0.1f * (float)(i % 3);
        pos[3 * i + 1] = (float)((i / 4) % 4) * 2.5f;
        pos[3 * i + 2] = (float)(i / 16) * 2.5f;
        h[i] = 3.0f;
        mu[i] = 1e19f;
        nH[i] = 1e-2f;
        T[i] = 1e4f;
        x[i] = 0.5;
    }
    int64_t src[3] = {0, 17, 63}, cnt[3 * NR], off[3 * NR];
    double Ncol[3 * NR];
    CHECK(orc_columns(N, pos, h, mu, x, NR, dirs, 10.0, 10.0, 3, src, 1e-12, 0, NULL, cnt, NULL,
                      NULL, NULL, NULL, 1) == 0);
    int64_t tot = 0;
    for (int r = 0; r < 3 * NR; ++r) {
        off[r] = tot;
        tot += cnt[r];
    }
    CHECK(tot > 0);
    int32_t* hj = malloc(sizeof(int32_t) * tot);
    int32_t* hi = malloc(sizeof(int32_t) * tot);
    double* hf = malloc(sizeof(double) * tot);
    CHECK(orc_columns(N, pos, h, mu, x, NR, dirs, 10.0, 10.0, 3, src, 1e-12, 1, Ncol, NULL, off,
                      hj, hi, hf, 1) == 0);
    for (int r = 0; r < 3 * NR; ++r) CHECK(isfinite(Ncol[r]) && Ncol[r] > 0.0);
    double sig[2] = {6.3e-18, 3e-18}, w[2] = {1e5, 2e5}, lnG[3], G[3], tau[3];
    orc_gamma(3, NR, Ncol, 2, sig, w, lnG, G, tau);
    for (int i = 0; i < 3; ++i) CHECK(isfinite(lnG[i]));
    double xh[3 * N], lh[2 * N], md[2];
    int32_t it = 0;
    CHECK(orc_solve(N, pos, h, mu, nH, T, NR, dirs, 2, sig, w, 10.0, 10.0, 0.0, 2, NULL, 1e-10,
                    1, xh, lh, NULL, &it, md) == 0);
    CHECK(it == 2);
    int32_t perm[N], skip[2 * N], first[2 * N], count[2 * N], root[3], end[3];
    uint64_t codes[N];
    float lo[6 * N], hi2[6 * N];
    CHECK(orc_lbvh(N, pos, h, 4, perm, codes, lo, hi2, skip, first, count) > 0);
    int64_t hoff[4] = {0, 10, 11, N};
    CHECK(orc_lbvh_seg(N, pos, h, 4, 3, hoff, perm, codes, lo, hi2, skip, first, count, root,
                       end) > 0);
    for (int g = 0; g < 3; ++g) CHECK(root[g] >= 0 && end[g] > root[g]);
    CHECK(isfinite(orc_slab_lnG(log(1e-12), 1e-2, 4e-13, 6e-16, 6.3e-18, 1e20)));
    CHECK(isfinite(orc_slab_lnG_poly(2, sig, w, 1e17, 1e-2, 4e-13, 6e-16, 1e20)));
    free(hj);
    free(hi);
    free(hf);
    printf("oracle checks passed\n");
    return 0;
}
