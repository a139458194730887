/*
 * CPU oracle for FNT-CDC + FNT-AEQ -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path never calls it and shares no code
 * with it.
 *
 * It computes, by the plain definitions and with no transform, blocking or
 * fusion, the exact integer results that the Fermat-number-transform path of
 * the paper must reproduce:
 *
 *  - CDC (Proposed FNT-CDC&AEQ structure, Eqs. (5), (7), (8) and Fig. 2):
 *    the causal linear convolution of the complex 5-bit dual-polarisation
 *    stream with the complex 6-bit CD-inverse taps, exactly, over the
 *    Gaussian integers.  Overlap-save with zero padding (the remark after
 *    Eq. (5)) and the complex packing of Eqs. (7)-(8) reach exactly this when
 *    Eq. (5) holds, which it does for 5-bit data and <= 32 taps of 6 bit.
 *  - Resampling to 1 sample/symbol (Experimental verification section) and
 *    requantisation to the 5-bit AEQ input width (parameters of the AEQ).
 *  - AEQ (4x4 real-valued MIMO, RDE tap update of Eq. (6), 14-bit taps):
 *    direct real FIRs per block of 16 symbols, then the block tap update.
 *
 * Where the paper is silent (rounding, saturation, RDE radii, step-size
 * shifts, block cadence) this file fixes the following integer forms:
 *   rs(v, s)  = floor((v + 2^(s-1)) / 2^s) for s >= 1, rs(v, 0) = v
 *   sat_b(v)  = clamp(v, -2^(b-1), 2^(b-1) - 1)
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_AEQ_TAPS 16
#define ORC_AEQ_BLOCK 16
#define ORC_CDC_HIST 32

/* floor(a / b) for b > 0, written out so it does not depend on how C rounds. */
static int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    int64_t r = a % b;
    if (r != 0 && a < 0) q -= 1;
    return q;
}

/* Round half up, then drop s fraction bits. */
static int64_t rs(int64_t v, int s) {
    if (s <= 0) return v;
    int64_t p = (int64_t)1 << s;
    return floor_div(v + p / 2, p);
}

static int64_t sat(int64_t v, int bits) {
    int64_t hi = ((int64_t)1 << (bits - 1)) - 1;
    int64_t lo = -((int64_t)1 << (bits - 1));
    if (v > hi) return hi;
    if (v < lo) return lo;
    return v;
}

/* ------------------------------------------------------------------ CDC -- */

/* Sample component c of instant i, with i < 0 reaching into the history
 * (hist[ORC_CDC_HIST-1] is the instant right before in[0]); zero if none. */
static int cdc_sample(const int8_t *in, const int8_t *hist, int64_t i, int c) {
    if (i >= 0) return in[i * 4 + c];
    if (hist && i >= -ORC_CDC_HIST) return hist[(ORC_CDC_HIST + i) * 4 + c];
    return 0;
}

/*
 * in      int8 [n][4]  {XI, XQ, YI, YQ}, 5-bit values at 2 samples/symbol
 * taps    int8 [L][2]  (re, im), 6-bit values
 * hist    int8 [32][4] the 32 instants preceding in[0], or NULL for zeros
 * z_out   int32 [n][4] exact convolution {Re zX, Im zX, Re zY, Im zY}, or NULL
 * a_out   int8 [M][4]  sat5(rs(z[2m+phase], shift)), M = (n + 1 - phase) / 2, or NULL
 */
void orc_cdc(const int8_t *in, int64_t n, const int8_t *taps, int L, int shift,
             int phase, const int8_t *hist, int32_t *z_out, int8_t *a_out) {
    for (int64_t i = 0; i < n; ++i) {
        int64_t z[4];
        for (int p = 0; p < 2; ++p) {
            int64_t re = 0, im = 0;
            for (int k = 0; k < L; ++k) {
                int64_t hr = taps[2 * k], hi = taps[2 * k + 1];
                int64_t xr = cdc_sample(in, hist, i - k, 2 * p);
                int64_t xi = cdc_sample(in, hist, i - k, 2 * p + 1);
                re += hr * xr - hi * xi;   /* (hr + j hi)(xr + j xi) */
                im += hr * xi + hi * xr;
            }
            z[2 * p] = re;
            z[2 * p + 1] = im;
        }
        if (z_out)
            for (int c = 0; c < 4; ++c) z_out[i * 4 + c] = (int32_t)z[c];
        if (a_out && i >= phase && ((i - phase) % 2) == 0) {
            int64_t m = (i - phase) / 2;
            for (int c = 0; c < 4; ++c) a_out[m * 4 + c] = (int8_t)sat(rs(z[c], shift), 5);
        }
    }
}

/* ------------------------------------------------------------------ AEQ -- */

typedef struct orc_aeq_params {
    int32_t out_shift;     /* s_o : y -> yhat */
    int32_t err_shift;     /* s_e : e * yhat -> 8-bit error term */
    int32_t mu_shift;      /* s_mu: gradient -> tap increment (mu = 2^-(s_e+s_mu)) */
    int32_t const_unit;    /* c_y : 16QAM unit amplitude at the output */
    int32_t update_enable; /* 0: fixed filter bank */
    /* Step schedule: the block with stream index j = block0 + (its index in this
     * call) updates with s_mu = mu_shift while j < gear_blocks and with
     * mu_shift_late from then on; gear_blocks = 0: mu_shift throughout. */
    int32_t mu_shift_late;
    int32_t gear_blocks;
    int64_t block0;
} orc_aeq_params;

static int aeq_sample(const int8_t *a, const int8_t *hist, int64_t m, int s) {
    if (m >= 0) return a[m * 4 + s];
    if (hist && m >= -ORC_AEQ_TAPS) return hist[(ORC_AEQ_TAPS + m) * 4 + s];
    return 0;
}

/*
 * a     int8 [M][4] 1 sample/symbol {XI, XQ, YI, YQ}, 5-bit
 * w     int16 [4 S1][4 S2][16] taps, 14-bit; updated in place (final state)
 * hist  int8 [16][4] the 16 symbols preceding a[0], or NULL for zeros
 * out   int16 [M][4] yhat
 */
void orc_aeq(const int8_t *a, int64_t M, int16_t *w, const orc_aeq_params *p,
             const int8_t *hist, int16_t *out) {
    int64_t c2 = (int64_t)p->const_unit * p->const_unit;
    for (int64_t b0 = 0; b0 < M; b0 += ORC_AEQ_BLOCK) {
        int64_t b1 = b0 + ORC_AEQ_BLOCK < M ? b0 + ORC_AEQ_BLOCK : M;
        int64_t eps[ORC_AEQ_BLOCK][4];
        for (int64_t m = b0; m < b1; ++m) {
            int64_t yh[4];
            /* 4x4 real-valued MIMO: 16 real FIRs, one per (S1, S2) pair */
            for (int s2 = 0; s2 < 4; ++s2) {
                int64_t y = 0;
                for (int s1 = 0; s1 < 4; ++s1)
                    for (int k = 0; k < ORC_AEQ_TAPS; ++k)
                        y += (int64_t)w[(s1 * 4 + s2) * ORC_AEQ_TAPS + k] *
                             aeq_sample(a, hist, m - k, s1);
                yh[s2] = sat(rs(y, p->out_shift), 16);
                out[m * 4 + s2] = (int16_t)yh[s2];
            }
            /* radius-directed error per polarisation, 16QAM rings 2, 10, 18 */
            for (int pol = 0; pol < 2; ++pol) {
                int64_t yi = yh[2 * pol], yq = yh[2 * pol + 1];
                int64_t r2 = yi * yi + yq * yq;
                int64_t R2 = r2 < 6 * c2 ? 2 * c2 : (r2 < 14 * c2 ? 10 * c2 : 18 * c2);
                int64_t e = R2 - r2;
                eps[m - b0][2 * pol] = sat(rs(e * yi, p->err_shift), 8);
                eps[m - b0][2 * pol + 1] = sat(rs(e * yq, p->err_shift), 8);
            }
        }
        if (!p->update_enable) continue;
        const int64_t j = p->block0 + b0 / ORC_AEQ_BLOCK;
        const int mu = (p->gear_blocks > 0 && j >= p->gear_blocks) ? p->mu_shift_late : p->mu_shift;
        /* Eq. (6) summed over the block: w_{S1-S2} += mu * e_S2 * in_S1 * out_S2 */
        for (int s1 = 0; s1 < 4; ++s1)
            for (int s2 = 0; s2 < 4; ++s2)
                for (int k = 0; k < ORC_AEQ_TAPS; ++k) {
                    int64_t g = 0;
                    for (int64_t m = b0; m < b1; ++m)
                        g += eps[m - b0][s2] * aeq_sample(a, hist, m - k, s1);
                    int16_t *wp = &w[(s1 * 4 + s2) * ORC_AEQ_TAPS + k];
                    *wp = (int16_t)sat((int64_t)*wp + rs(g, mu), 14);
                }
    }
}

/* ------------------------------------------------------------ CDC + AEQ -- */

/*
 * The receiver chain on one channel: CDC at 2 sps, resample + requantise,
 * AEQ at 1 sps.  a_buf is caller scratch of M*4 bytes (M = (n+1-phase)/2).
 */
void orc_cdc_aeq(const int8_t *in, int64_t n, const int8_t *taps, int L, int shift,
                 int phase, const int8_t *cdc_hist, int16_t *w,
                 const orc_aeq_params *p, const int8_t *aeq_hist, int8_t *a_buf,
                 int16_t *out) {
    int64_t M = (n + 1 - phase) / 2;
    if (n <= 0 || M <= 0) return;
    orc_cdc(in, n, taps, L, shift, phase, cdc_hist, NULL, a_buf);
    orc_aeq(a_buf, M, w, p, aeq_hist, out);
}

/* One independent channel of a batch. */
typedef struct orc_channel {
    const int8_t *in;
    int64_t n;
    const int8_t *taps;   /* [L][2] */
    int32_t ntaps;
    int32_t shift;
    int32_t phase;
    int32_t pad_;
    int16_t *w;           /* [256], in/out */
    int8_t *a_buf;        /* scratch [M][4] */
    int16_t *out;         /* [M][4] */
    orc_aeq_params aeq;
} orc_channel;

/* Run many channels; OpenMP over channels when threads > 1.  Returns the
 * number of threads actually used. */
int orc_batch(orc_channel *ch, int64_t nch, int threads) {
    int used = 1;
#ifdef _OPENMP
    if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
    for (int64_t c = 0; c < nch; ++c) {
        if (c == 0) used = omp_get_num_threads();
        orc_cdc_aeq(ch[c].in, ch[c].n, ch[c].taps, ch[c].ntaps, ch[c].shift, ch[c].phase,
                    NULL, ch[c].w, &ch[c].aeq, NULL, ch[c].a_buf, ch[c].out);
    }
#else
    (void)threads;
    for (int64_t c = 0; c < nch; ++c)
        orc_cdc_aeq(ch[c].in, ch[c].n, ch[c].taps, ch[c].ntaps, ch[c].shift, ch[c].phase,
                    NULL, ch[c].w, &ch[c].aeq, NULL, ch[c].a_buf, ch[c].out);
#endif
    return used;
}

/* Exposed helpers so the rounding rules can be pinned by tests. */
int64_t orc_rs(int64_t v, int s) { return rs(v, s); }
int64_t orc_sat(int64_t v, int bits) { return sat(v, bits); }
