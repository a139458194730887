/* Drives every function of the oracle (oracle/oracle.c, included here) over
 * edge cases, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py): empty, one-sample and ragged streams, both
 * decimation phases, with and without histories, 1 to 65 taps, the extreme
 * shifts and constant, saturating taps and inputs, and the OpenMP batch.  The
 * sanitizers abort on the first finding; a clean run prints "ok". */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.c"

static uint64_t rng_state = 88172645463325252ull;
static int64_t rnd(int64_t lo, int64_t hi) {    /* xorshift64, inclusive range */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return lo + (int64_t)(rng_state % (uint64_t)(hi - lo + 1));
}

static int8_t *samples(int64_t n, int extreme) {
    int8_t *x = (int8_t *)malloc((size_t)(n > 0 ? n : 1) * 4);
    for (int64_t i = 0; i < 4 * n; ++i) x[i] = (int8_t)(extreme ? -16 : rnd(-16, 15));
    return x;
}

int main(void) {
    const int64_t lengths[] = {0, 1, 2, 31, 32, 33, 63, 64, 65, 1000, 4099};
    const int ntaps[] = {1, 8, 32, 33, 65};
    const orc_aeq_params prms[] = {{7, 16, 3, 52, 1}, {24, 62, 40, 4096, 1}, {0, 0, 0, 1, 1},
                                   {12, 30, 9, 1, 1}, {9, 12, 1, 33, 0}};
    int8_t hist_cdc[32 * 4], hist_aeq[16 * 4];
    for (int i = 0; i < 32 * 4; ++i) hist_cdc[i] = (int8_t)rnd(-16, 15);
    for (int i = 0; i < 16 * 4; ++i) hist_aeq[i] = (int8_t)rnd(-16, 15);
    for (size_t li = 0; li < sizeof lengths / sizeof *lengths; ++li) {
        const int64_t n = lengths[li];
        for (int ex = 0; ex < 2; ++ex) {
            int8_t *x = samples(n, ex);
            for (size_t ti = 0; ti < sizeof ntaps / sizeof *ntaps; ++ti) {
                const int L = ntaps[ti];
                int8_t taps[65 * 2];
                for (int k = 0; k < 2 * L; ++k) taps[k] = (int8_t)(ex ? -32 : rnd(-32, 31));
                for (int phase = 0; phase < 2; ++phase) {
                    const int64_t M = n + 1 > phase ? (n + 1 - phase) / 2 : 0;
                    int32_t *z = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * 16);
                    int8_t *a = (int8_t *)malloc((size_t)(M > 0 ? M : 1) * 4);
                    int16_t *out = (int16_t *)malloc((size_t)(M > 0 ? M : 1) * 8);
                    const int shift = (int)rnd(0, 16);
                    orc_cdc(x, n, taps, L, shift, phase, (L <= 33 && (li & 1)) ? hist_cdc : NULL, z, a);
                    orc_cdc(x, n, taps, L, shift, phase, NULL, NULL, a);
                    orc_cdc(x, n, taps, L, shift, phase, NULL, z, NULL);
                    for (size_t pi = 0; pi < sizeof prms / sizeof *prms; ++pi) {
                        int16_t w[256];
                        for (int k = 0; k < 256; ++k) w[k] = (int16_t)(ex ? (k & 1 ? 8191 : -8192) : rnd(-8192, 8191));
                        orc_aeq(a, M, w, &prms[pi], (pi & 1) ? hist_aeq : NULL, out);
                        int8_t abuf[4 * 2100];
                        if (M <= 2100 && L <= 33)
                            orc_cdc_aeq(x, n, taps, L, shift, phase, (pi & 1) ? hist_cdc : NULL, w, &prms[pi],
                                        (pi & 1) ? hist_aeq : NULL, abuf, out);
                    }
                    free(z);
                    free(a);
                    free(out);
                }
            }
            free(x);
        }
    }
    /* the OpenMP batch over channels of mixed lengths */
    enum { NCH = 12 };
    orc_channel ch[NCH];
    int8_t taps[NCH][32 * 2];
    for (int c = 0; c < NCH; ++c) {
        const int64_t n = lengths[c % 11];
        const int64_t M = (n + 1) / 2;
        for (int k = 0; k < 64; ++k) taps[c][k] = (int8_t)rnd(-32, 31);
        ch[c].in = samples(n, 0);
        ch[c].n = n;
        ch[c].taps = taps[c];
        ch[c].ntaps = 1 + c % 32;
        ch[c].shift = c % 9;
        ch[c].phase = 0;
        ch[c].pad_ = 0;
        ch[c].w = (int16_t *)calloc(256, sizeof(int16_t));
        for (int q = 0; q < 4; ++q) ch[c].w[q * 64 + q * 16 + 8] = 4096;
        ch[c].a_buf = (int8_t *)malloc((size_t)(M > 0 ? M : 1) * 4);
        ch[c].out = (int16_t *)malloc((size_t)(M > 0 ? M : 1) * 8);
        ch[c].aeq = prms[c % 5];
    }
    const int used = orc_batch(ch, NCH, 4);
    for (int c = 0; c < NCH; ++c) {
        free((void *)ch[c].in);
        free(ch[c].w);
        free(ch[c].a_buf);
        free(ch[c].out);
    }
    /* the rounding helpers at the widths the definitions use */
    const int64_t vs[] = {0, 1, -1, 127, -128, (int64_t)1 << 40, -((int64_t)1 << 40), (int64_t)1 << 50};
    int64_t acc = 0;
    for (size_t i = 0; i < sizeof vs / sizeof *vs; ++i)
        for (int s = 0; s <= 62; ++s) acc += orc_rs(vs[i], s) + orc_sat(vs[i], 1 + s % 32);
    printf("ok %d %lld\n", used, (long long)acc);
    return 0;
}
