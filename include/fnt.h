/*
 * libfnt -- Fermat-number-transform chromatic-dispersion compensation (FNT-CDC)
 * and adaptive equalisation (FNT-AEQ) on AMD MI355X (gfx950).
 *
 * Method: "Fermat Number Transform Based Chromatic Dispersion Compensation and
 * Adaptive Equalization Algorithm" (arXiv 2405.04253).
 *
 * Conventions for every entry point
 *  - Return value: FNT_OK (0) or one of the FNT_E_* codes below.  No exception,
 *    abort or longjmp crosses this interface.  fnt_last_error() gives text for the
 *    last failure on the calling thread.
 *  - Buffers are caller-owned DEVICE pointers unless a name starts with host_.
 *    The library never frees caller memory.  int8 sample/symbol buffers must be
 *    4-byte aligned, int16/int32 buffers 8-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    that take a stream only enqueue work on it and return; results are valid
 *    once the stream has reached that point.
 *  - Values that must lie in a declared bit width and live in device memory are
 *    checked by the kernels; a violation is latched in a per-device flag and
 *    reported as FNT_E_RANGE by fnt_check().  Outputs of such a call are then
 *    unspecified (but every access stays in bounds).
 *
 * Data layouts
 *  - instant   : one 2-samples/symbol dual-polarisation sample, int8[4] =
 *                {XI, XQ, YI, YQ}, each 5-bit two's complement in [-16, 15].
 *  - symbol    : one 1-sample/symbol dual-polarisation value, int8[4] (AEQ
 *                input, 5 bit) or int16[4] (AEQ output).
 *  - AEQ taps  : int16[4 S1][4 S2][16], 14-bit two's complement in
 *                [-8192, 8191]; S1 = input stream, S2 = output stream, both
 *                ordered XI, XQ, YI, YQ (4x4 real-valued MIMO).
 */
#ifndef FNT_H
#define FNT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FNT_OK = 0,
    FNT_E_INVAL = 1,   /* bad shape, parameter, alignment or NULL pointer */
    FNT_E_RANGE = 2,   /* an input value outside its declared bit width / >= F */
    FNT_E_NOMEM = 3,   /* device or host allocation failed */
    FNT_E_DEVICE = 4,  /* a HIP call failed (text in fnt_last_error) */
    FNT_E_BUSY = 5,    /* admission refused: the request does not fit right now */
    FNT_E_STATE = 6    /* unknown channel / ticket, or an object in the wrong state */
};

enum { FNT_ALPHA_2 = 0, FNT_ALPHA_SQRT2 = 1 };

#define FNT_MAX_CDC_TAPS 32
/* Taps of fnt_cdc_long: overlap-save with N = 128 and 64 new instants per block. */
#define FNT_MAX_CDC_LONG_TAPS 65
#define FNT_AEQ_TAPS 16
#define FNT_AEQ_BLOCK 16       /* symbols per AEQ block (one tap update per block) */
#define FNT_CDC_HOP 32         /* new instants per CDC overlap-save block */

/* Text of the last error on this thread ("" if none).  The pointer stays valid
 * until the next failing call on the same thread. */
const char *fnt_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int fnt_version(void);

/* Synchronise `stream`, then report and clear the per-device range flag of the
 * current device: FNT_E_RANGE if any kernel launched since the previous check
 * saw an out-of-range input; FNT_E_DEVICE if a bounded wait inside a fused
 * launch (fnt_cdc_aeq, fused plans) gave up, which a correct launch never does
 * (that launch's outputs are then unspecified); else FNT_OK. */
int fnt_check(void *stream);

/* ------------------------------------------------------------------------
 * Transforms -- Eq. (1) (forward) and Eq. (2) (inverse, including N^-1) over
 * Z_F with F = 2^(2^t) + 1 (FNT section), t in {2, 3, 4}, N the order of the
 * radix (Eq. (4) with alpha^(N/2) = -1): N = 2^(t+1) for alpha = 2 and
 * N = 2^(t+2) for alpha = sqrt 2 = 2^(3q/4) - 2^(q/4), q = 2^t (6 mod 17,
 * 60 mod 257, 4080 mod 65537).  Among them:
 *   (2,  8, 2)      the 8-point, radix-2, modulus-17 example of Fig. 1
 *   (4, 32, 2)      the FNT-AEQ transform (Proposed structure, AEQ part)
 *   (4, 64, sqrt 2) the FNT-CDC transform (Proposed structure, CDC part),
 *                   alpha = 2^12 - 2^4 = 4080, the square root of 2 whose
 *                   powers are sums of two powers of two
 *   (2, 16, sqrt 2), (3, 16, 2), (3, 32, sqrt 2): the same construction over
 *                   the smaller Fermat primes, for narrower word widths.
 * x, X : uint32[batch][N], natural order, canonical residues in [0, F).  In-place
 * (x == X) is allowed.  Inputs >= F are a range error (flagged, see fnt_check).
 * log2n must equal log2 of N above; other combinations return FNT_E_INVAL.
 * ------------------------------------------------------------------------ */
int fnt_forward(const uint32_t *x, uint32_t *X, size_t batch, int t, int log2n,
                int alpha_kind, void *stream);
int fnt_inverse(const uint32_t *X, uint32_t *x, size_t batch, int t, int log2n,
                int alpha_kind, void *stream);

/* ------------------------------------------------------------------------
 * Parameters (host structs, copied at call time)
 * ------------------------------------------------------------------------ */

/* CDC (Proposed structure: F = 65537, alpha = sqrt 2, N = 64, 5-bit signal,
 * 6-bit taps; complex product by Eqs. (7)-(8)).
 *   taps[k] = (re, im), 6-bit in [-32, 31], k < ntaps; entries >= ntaps ignored.
 *   ntaps in [1, 32]: with 32 new instants per 64-point block the circular
 *   convolution equals the linear one (the zero-padding remark after Eq. (5)),
 *   and Eq. (5) holds: 32 taps * 1024 <= (F - 1) / 2.
 *   requant_shift s_c in [0, 16]: the 1-sample/symbol output is
 *   a[m] = sat5(rs(z[2m + decim_phase], s_c)), rs(v, s) = floor((v + 2^(s-1)) / 2^s).
 *   decim_phase in {0, 1}: which 2-sps instant of each symbol is kept. */
typedef struct fnt_cdc_params {
    int8_t taps[FNT_MAX_CDC_TAPS][2];
    int32_t ntaps;
    int32_t requant_shift;
    int32_t decim_phase;
} fnt_cdc_params;

/* AEQ (4x4 real-valued MIMO with the RDE update of Eq. (6); 14-bit taps split
 * into two 7-bit groups convolved separately through F = 65537, alpha = 2,
 * N = 32 transforms).  Per block of 16 symbols, with the block's taps w:
 *   y_S2[m]  = sum_S1 sum_k w[S1][S2][k] * a_S1[m - k]           (exact)
 *   yhat     = sat16(rs(y, out_shift))                              -> output
 *   r2_P     = yhat_PI^2 + yhat_PQ^2,  R2 = c^2 * {2 if r2 < 6c^2, 10 if r2 < 14c^2, else 18}
 *   eps_S2   = sat8(rs((R2 - r2_pol(S2)) * yhat_S2, err_shift))
 *   w       <- sat14(w + rs(sum_m eps_S2[m] * a_S1[m - k], s_mu))   if update_enable
 * Step schedule: s_mu = mu_shift for the blocks of a stream with index below
 * gear_blocks (counted from the stream's first block, across session segments)
 * and mu_shift_late from then on; gear_blocks = 0: mu_shift throughout (a
 * large step to converge, then a small one for a low floor).
 *   out_shift in [0, 24], err_shift in [0, 62], mu_shift and mu_shift_late in
 *   [0, 40], const_unit c in [1, 4096], update_enable in {0, 1}. */
typedef struct fnt_aeq_params {
    int32_t out_shift;
    int32_t err_shift;
    int32_t mu_shift;
    int32_t const_unit;
    int32_t update_enable;
    int32_t mu_shift_late;
    uint32_t gear_blocks;
} fnt_aeq_params;

/* ------------------------------------------------------------------------
 * Single-stream calls (zero history before the first sample).
 * ------------------------------------------------------------------------ */

/* FNT-CDC of n instants (Fig. 2 structure, Eqs. (5), (7), (8)).
 *   in        int8[n][4] device
 *   out_exact int32[n][4] device or NULL: exact z = {Re zX, Im zX, Re zY, Im zY}
 *   out_1sps  int8[M][4] device or NULL, M = (n + 1 - decim_phase) / 2:
 *             resampled to 1 sample/symbol and requantised to 5 bit. */
int fnt_cdc(const int8_t *in, uint64_t n, const fnt_cdc_params *p, int32_t *out_exact,
            int8_t *out_1sps, void *stream);

/* FNT-CDC with a longer transform, for 1 .. 65 taps (the N = 64 block of
 * fnt_cdc holds 33): N = 128, 64 new instants per block, radix 4938 of order
 * 128 modulo 65537 (a square root of the CDC's sqrt 2).  A 65-tap convolution
 * leaves the Eq. (5) bound (65 * 1008 = 65520 > 32768), so the 6-bit taps are
 * split into balanced 3-bit digits, h = 8 hi + lo (lo in [-4, 3]); each digit
 * is convolved through the packing of Eqs. (7)-(8) (within 65 * 128 = 8320) and
 * the centred results are combined as 8 z_hi + z_lo.  Same results as the
 * direct convolution (zero history before in[0]).
 *   in         int8[n][4] device
 *   host_taps  int8[ntaps][2] host memory, (re, im) in [-32, 31]; read during the call
 *   out_exact  int32[n][4] device or NULL (16-byte aligned)
 *   out_1sps   int8[M][4] device or NULL, M = (n + 1 - decim_phase) / 2.
 * FNT_E_INVAL for ntaps outside 1 .. 65, requant_shift outside 0 .. 16, a phase
 * other than 0 or 1, a NULL or misaligned buffer; FNT_E_RANGE for a tap outside
 * 6 bit (nothing launched); samples outside 5 bit are latched for fnt_check. */
int fnt_cdc_long(const int8_t *in, uint64_t n, const int8_t *host_taps, int ntaps, int requant_shift,
                 int decim_phase, int32_t *out_exact, int8_t *out_1sps, void *stream);

/* FNT-AEQ of m symbols (Fig. 3 structure, Eq. (6)).
 *   in_1sps int8[m][4] device (5-bit values)
 *   taps    int16[4][4][16] device, read at the start, overwritten with the state
 *           after the last block's update
 *   out     int16[m][4] device.
 * The final partial block (m not a multiple of 16) updates from its valid
 * symbols only. */
int fnt_aeq(const int8_t *in_1sps, uint64_t m, int16_t *taps, const fnt_aeq_params *p,
            int16_t *out, void *stream);

/* The receiver chain on one channel (experimental section: CDC, resampling to
 * 1 sample/symbol, then the AEQ; Figs. 2 and 3): the same results as fnt_cdc to
 * the 1-sample/symbol stream followed by fnt_aeq, in ONE kernel launch that
 * allocates nothing.  Inside the launch one wave computes the CDC 64 blocks at a
 * time into a ring in on-chip memory (LDS) while the AEQ chain consumes it, so
 * the 1-sample/symbol stream never goes to device memory.
 *   in   int8[n][4] device;  taps as for fnt_aeq (in/out);
 *   out  int16[M][4] device with M = (n + 1 - decim_phase) / 2. */
int fnt_cdc_aeq(const int8_t *in, uint64_t n, const fnt_cdc_params *cp, int16_t *taps,
                const fnt_aeq_params *ap, int16_t *out, void *stream);

/* ------------------------------------------------------------------------
 * Batched plans: many independent channels in one launch sequence.
 * ------------------------------------------------------------------------ */

typedef struct fnt_channel_desc {
    const int8_t *in;      /* device int8[n][4] */
    int16_t *out;          /* device int16[M][4], M = (n + 1 - cdc.decim_phase) / 2 */
    int16_t *taps;         /* device int16[4][4][16], in/out as for fnt_aeq */
    uint64_t n;            /* instants */
    fnt_cdc_params cdc;
    fnt_aeq_params aeq;
} fnt_channel_desc;

typedef struct fnt_plan_config {
    int32_t device;        /* HIP device ordinal the buffers live on */
    int32_t autotune;      /* 1: time the candidate schedules at create and keep the fastest */
    int32_t use_graph;     /* 1: capture the launch sequence in a hipGraph, replay it in run */
    int32_t tune_quick;    /* with autotune: 1 = a short candidate list (the lane-per-block CDC
                              groupings, three leads, the fused schedules), for batches whose
                              every run takes long; 0 = the full sweep */
    const char *tune_cache;/* optional JSON file remembering autotune results (NULL: none) */
} fnt_plan_config;

typedef struct fnt_plan_info {
    uint64_t channels;
    uint64_t instants;     /* total instants over all channels */
    uint64_t symbols;      /* total output symbols */
    uint64_t cdc_blocks;   /* total 32-instant CDC blocks */
    uint64_t aeq_blocks_max;  /* longest per-channel AEQ chain, in 16-symbol blocks */
    int32_t cdc_waves_per_group;  /* chosen schedule */
    int32_t cdc_blocks_per_wave;  /* 0 = one block per lane (64 blocks per wave) */
    int32_t aeq_variant;   /* 0 = Fermat-domain filtering (the method), 1 = direct comparator,
                              2 = Fermat-domain, one wave per channel, 3 = the same with the
                              RDE gradient in the Fermat domain too */
    int32_t aeq_waves_per_pol;  /* variant 0: AEQ form (0, 3, 1, 5, 2, 4; see fnt_plan_set_aeq_waves) */
    int32_t graph;         /* 1 if fnt_plan_run replays a hipGraph (plans created with use_graph) */
    int32_t aeq_waves_long;     /* AEQ form of the long chains (see fnt_plan_set_aeq_split) */
    double tune_ms;        /* AEQ time of the chosen schedule during autotune, ms (0 if none) */
    uint64_t aeq_long_channels; /* longest channels run in their own concurrent launch */
    int32_t cdc_variant;   /* 0 = Fermat-domain (the method), 1 = direct comparator */
    int32_t lead_channels; /* pipelined lead channels in effect, first level included
                              (see fnt_plan_set_lead) */
    int32_t lead_form;     /* AEQ form of the lead channels after the first level */
    int32_t top_channels;  /* channels of the lead's first level (0: one level) */
    int32_t top_form;      /* AEQ form of the first level */
    double tune_run_ms;    /* whole-run time (CDC + AEQ) of the chosen schedule during autotune,
                              ms (0 if none) */
    int32_t fused_lpt;     /* 0: the staged / lead schedule above; 4, 8, 16: every run is one launch
                              of the fused kernel with that many AEQ lanes per transform (see
                              fnt_plan_set_fused) */
    int32_t fused_grid;    /* workgroups of the fused launch (0 when not fused) */
    uint64_t fused_prio_channels;  /* longest channels at raised wave priority in the fused launch */
    int32_t fused_split;   /* 1: the fused launch runs one workgroup per polarisation half */
    int32_t reserved2;
} fnt_plan_info;

typedef struct fnt_plan fnt_plan;

/* Build a plan for `nch` channels (copied; the device buffers must stay valid
 * while the plan is used).  Allocates the plan's device tables and scratch.
 * With autotune, times the candidate CDC schedules and AEQ schedules (waves per
 * half, split of the longest chains) on `stream`: the CDC runs write plan
 * scratch, the AEQ runs work on scratch copies of the taps and write `out`
 * (which a real run overwrites); the caller's taps are not touched. */
int fnt_plan_create(fnt_plan **plan, const fnt_channel_desc *host_channels, size_t nch,
                    const fnt_plan_config *cfg, void *stream);
/* Run every channel once (CDC + resample + AEQ), enqueued on `stream`. */
int fnt_plan_run(fnt_plan *plan, void *stream);
/* The run as a replay of the plan's captured hipGraph (what fnt_plan_run does
 * for plans created with use_graph).  With a pipelined lead the graph has the
 * lead's branch on its own stream, forked and joined by events inside the
 * capture.  FNT_E_STATE if the plan has no graph (created without use_graph). */
int fnt_plan_run_graph(fnt_plan *plan, void *stream);

#define FNT_STAGE_CDC 1   /* CDC + resample + requantise of every channel (writes plan scratch) */
#define FNT_STAGE_AEQ 2   /* AEQ of every channel (reads plan scratch, updates taps, writes out) */
#define FNT_STAGE_ALL 3
/* Launch the stages in `stages` (a mask of FNT_STAGE_*) directly on `stream`,
 * outside the plan's graph, so that a caller can bracket each with its own
 * events.  FNT_STAGE_CDC then FNT_STAGE_AEQ computes exactly what one
 * fnt_plan_run does (the stages never pipeline a lead, fnt_plan_set_lead); the
 * AEQ stage alone recomputes the AEQ from whatever the last CDC stage left in
 * the scratch (taps continue from their current state).  FNT_E_INVAL for a
 * mask outside FNT_STAGE_ALL. */
int fnt_plan_run_stage(fnt_plan *plan, int stages, void *stream);
int fnt_plan_get_info(const fnt_plan *plan, fnt_plan_info *info);
int fnt_plan_destroy(fnt_plan *plan);

/* Select the AEQ kernel of a plan: 0 = Fermat-domain filtering split by output
 * polarisation (default, the method), 1 = direct time-domain comparator with
 * bit-identical results and no Fermat-domain arithmetic, 2 = Fermat-domain
 * filtering with one wave per channel, 3 = as 2 with the RDE gradient of the
 * tap update (Eq. (6)) also formed in the Fermat domain: a correlation of the
 * block's 8-bit error terms with the window through FNT32 products, exact
 * because its magnitude stays within the Eq. (5) bound (16 * 128 * 16 =
 * 32768); bit-identical results.  FNT_E_INVAL for another value. */
int fnt_plan_set_aeq_variant(fnt_plan *plan, int variant);
/* Form of AEQ variant 0 (the Fermat-domain method), from the fewest
 * instructions per block to the shortest serial latency per block:
 *   0: every lane runs whole transforms in its registers, 32 lanes per channel,
 *      two channels per wave;
 *   3: two lanes per transform, one channel per wave;
 *   1, 2, 4: split by output polarisation, that many waves per half, each half
 *      its own workgroup;
 *   5: split by output polarisation, one wave per half, both halves of a
 *      channel in one workgroup (the same arithmetic as 1).
 * Overrides the default / autotuned choice, including any split and lead. */
int fnt_plan_set_aeq_waves(fnt_plan *plan, int waves_per_pol);
/* Split the AEQ of a plan: the `long_channels` channels with the longest chains
 * run in form `wpp_long` (short serial latency, raised wave priority), the rest
 * in form `wpp` (fewer instructions per block); forms as for
 * fnt_plan_set_aeq_waves.  The pairs (1, 2, 4 or 5 with 0 or 3), (3, 0) and
 * (2, 5) run as one launch with the long chains' workgroups first; other pairs
 * as two concurrent launches.  long_channels = 0 disables the split. */
int fnt_plan_set_aeq_split(fnt_plan *plan, uint64_t long_channels, int wpp_long, int wpp);
/* Select the CDC kernel of a plan: 0 = overlap-save in the Fermat domain with the
 * complex product of Eqs. (7)-(8) (default, the method), 1 = direct time-domain
 * comparator (4-byte integer dot products over the 32-instant window, no
 * Fermat-domain arithmetic) with bit-identical results.  FNT_E_INVAL otherwise. */
int fnt_plan_set_cdc_variant(fnt_plan *plan, int variant);
/* CDC launch schedule: waves per workgroup (1, 2 or 4) and the block mapping.
 * blocks_per_wave = 0 (default): every lane transforms one whole 32-instant block
 * in its registers, a wave takes 64 consecutive blocks of one channel;
 * blocks_per_wave = 1 .. 1024: the lanes of a wave share one block at a time
 * (16 lanes per 64-point transform) and a wave takes that many consecutive
 * blocks.  Results do not depend on it. */
int fnt_plan_set_cdc_schedule(fnt_plan *plan, int waves_per_group, int blocks_per_wave);
/* Pipelined lead: the CDC of the `lead_channels` channels with the longest AEQ
 * chains runs first; their AEQ (in form `lead_form`, see fnt_plan_set_aeq_waves,
 * or the long chains' form for -1; at raised wave priority) then starts on the
 * plan's side stream while the CDC and the AEQ of the other channels run on the
 * launch stream, so the longest serial chains do not wait for the whole batch's
 * CDC.  lead_form 6: the lead channels' CDC and AEQ run together as one launch
 * of the fused kernel (see fnt_plan_set_fused; one wave per half) on the side
 * stream from the start, with no CDC launch of their own (no first level).  With 0 < top_channels < lead_channels the lead has two levels: the
 * `top_channels` longest run in form `top_form` (-1 as above).  If that form
 * pairs with the lead's in one split launch (see fnt_plan_set_aeq_split; e.g.
 * 2 with 5) they are the first workgroups of the lead's own launch; otherwise
 * their CDC runs first of all and their AEQ starts on a third stream, then the
 * CDC of the rest of the lead and its AEQ on the side stream.  The other channels keep the
 * split of fnt_plan_set_aeq_split for those of them among the long channels.
 * lead_channels = 0 (default unless the autotuner chose a lead) runs every CDC
 * before any AEQ.  In effect for 0 < lead_channels < channels when the other
 * channels' AEQ is one launch (no long channels left among them, a split that
 * runs as one launch, or an AEQ variant other than 0, whose forms are ignored);
 * otherwise the plan runs without a lead.  While a lead is in effect
 * fnt_plan_run launches the sequence directly instead of replaying the plan's
 * graph.  Results never depend on it.  Waits for the device to finish its
 * outstanding work (earlier runs may still read the plan's tables), then
 * rewrites the segmented CDC table.  FNT_E_INVAL for a NULL plan or another
 * form; FNT_E_NOMEM / FNT_E_DEVICE if the segmented CDC table cannot be
 * allocated / uploaded. */
int fnt_plan_set_lead(fnt_plan *plan, uint64_t lead_channels, int lead_form, uint64_t top_channels,
                      int top_form);

/* Fused persistent schedule: every fnt_plan_run is ONE launch of the fused
 * kernel (the receiver chain of the experimental section, Figs. 2 and 3):
 * each workgroup takes channels longest chain first from a work counter; per
 * channel one wave computes the CDC 64 blocks at a time into a ring in LDS
 * while the AEQ waves consume it, so the 1-sample/symbol stream never goes to
 * device memory and the longest chains start at once.  lpt = 4, 8 or 16 AEQ
 * lanes per transform (one, two or four waves per polarisation half; 4 suits
 * large batches, 16 the shortest serial latency), 0 switches the fused
 * schedule off (the staged / lead schedule applies again).  The
 * `prio_channels` longest channels run at raised wave priority.  Any other
 * schedule setter (fnt_plan_set_aeq_waves, _aeq_split, _lead, the variants)
 * switches it off.  split_halves = 1: one workgroup per polarisation half of
 * every channel, each computing the channel's CDC itself (twice the CDC work,
 * but each half's AEQ waves get a CU of their own: the shortest chains for a
 * few channels on an otherwise idle GPU); 0: both halves and one CDC per
 * workgroup, channels from a work counter.  Results never depend on it.
 * FNT_E_INVAL for another lpt or split_halves. */
int fnt_plan_set_fused(fnt_plan *plan, int lpt, uint64_t prio_channels, int split_halves);

typedef struct fnt_plan_timing {
    float step_ms;          /* first launch to the end of the last, on the launch stream */
    float cdc_ms;           /* the CDC launches, back to back on the launch stream */
    float aeq_ms;           /* the AEQ launch on the launch stream: the channels after the lead
                               (every channel without a lead) */
    float aeq_lead_ms;      /* the lead's AEQ launch on the side stream (after the first level;
                               0 without a lead) */
    uint64_t aeq_blocks;    /* 16-symbol AEQ blocks of the channels aeq_ms covers */
    uint64_t aeq_lead_blocks;  /* 16-symbol AEQ blocks of the channels aeq_lead_ms covers */
    float aeq_top_ms;       /* the first level's AEQ launch on the third stream (0 if none, or
                               if it runs inside the lead's launch) */
    int32_t fused;          /* 1: the run was one fused launch (aeq_ms is that launch, cdc_ms 0) */
    uint64_t aeq_top_blocks;   /* 16-symbol AEQ blocks of the first level's own launch */
} fnt_plan_timing;
/* Run every channel once, as fnt_plan_run does, but launch the sequence
 * directly (never the graph) with HIP events around every launch on the stream
 * it runs on; wait for the run to end and report the durations in `timing`
 * (caller-owned host struct).  Blocks the calling thread.  FNT_E_INVAL for NULL
 * arguments, FNT_E_DEVICE on a HIP error. */
int fnt_plan_run_timed(fnt_plan *plan, fnt_plan_timing *timing, void *stream);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under hipGraph stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the fused
 * run of fnt_plan_run (see fnt_plan_set_fused, one wave per polarisation half)
 * over up to FNT_NOALLOC_MAX_CHANNELS channels with NO allocation of any kind.
 * The device tables and the work counter that fnt_plan_create would allocate
 * live instead in a fixed device array of FNT_NOALLOC_SCRATCH_BYTES inside the
 * library, one per GPU, held until the process ends.
 *   dev_channels  fnt_channel_desc[nch] in DEVICE memory (8-byte aligned), each
 *                 as for fnt_plan_create (the buffers it names: device memory,
 *                 caller-owned); read on the device, so an invalid descriptor
 *                 is reported by fnt_check as FNT_E_INVAL and its channel is
 *                 skipped (nothing of it is read or written), the others run;
 *   nch           0 .. FNT_NOALLOC_MAX_CHANNELS; more returns FNT_E_INVAL.
 * Two kernel launches on `stream` (prepare, then fused); results as
 * fnt_plan_run's.  Every call on one GPU uses that GPU's one array and leaves
 * it to the next: calls that overlap on one GPU (different streams with no
 * ordering between them) race and must not be made.
 * ------------------------------------------------------------------------ */
#define FNT_NOALLOC_MAX_CHANNELS 4096
#define FNT_NOALLOC_SCRATCH_BYTES (1 << 20)
int fnt_cdc_aeq_batch_noalloc(const fnt_channel_desc *dev_channels, uint32_t nch, void *stream);

/* ------------------------------------------------------------------------
 * Serving sessions: continuing per-channel streams with device-resident state.
 * ------------------------------------------------------------------------ */

typedef struct fnt_session_config {
    int32_t device;
    uint32_t max_channels;     /* channel ids are 0 .. max_channels-1 */
    uint64_t hbm_budget_bytes; /* staging pool for FNT_SUBMIT_HOST requests + scratch */
    uint32_t chunk_blocks;     /* AEQ blocks advanced per request per tick (0: 512) */
    uint32_t max_active;       /* requests advanced per tick (0: max_channels) */
    int32_t aeq_form;          /* AEQ form of the ticks (see fnt_plan_set_aeq_waves), -1: by the
                                  number of requests in the tick (shortest tick for that load) */
    int32_t reserved;          /* 0 */
} fnt_session_config;

typedef struct fnt_session_stats {
    uint64_t submitted, completed, cancelled, rejected;
    uint64_t instants_done;    /* instants of completed requests */
    uint64_t ticks;            /* launch ticks issued */
    double p50_us, p99_us, mean_us, max_us;  /* completion - arrival, completed requests */
    double first_arrival_s, last_completion_s;  /* session clock, seconds */
    double gsamples_per_s;     /* instants_done / (last_completion - first_arrival) / 1e9 */
} fnt_session_stats;

typedef struct fnt_session fnt_session;

#define FNT_SUBMIT_HOST 1u     /* in/out are host pointers, staged through the HBM pool */

/* Session state of one channel, as exported by fnt_session_get_state. */
#define FNT_STATE_BYTES 768

uint64_t fnt_now_ns(void);     /* the session clock (monotonic, ns) */

int fnt_session_create(fnt_session **s, const fnt_session_config *cfg);
/* Register channel `ch` with its CDC and AEQ parameters and initial taps
 * (host int16[4][4][16]; NULL = centre spike 4096 at tap 8 on each S1 == S2). */
int fnt_session_add_channel(fnt_session *s, uint32_t ch, const fnt_cdc_params *cp,
                            const fnt_aeq_params *ap, const int16_t *host_init_taps);
/* Queue `n` instants (a multiple of 32) of channel `ch`'s continuing stream.
 * Output: n/2 symbols int16[n/2][4] (decim_phase 0) at `out`.  `in`/`out` are
 * device pointers unless flags has FNT_SUBMIT_HOST.  Requests of one channel run
 * in submission order; a channel's output depends only on its own stream.
 * arrival_ns (session clock, 0 = now) is the time latency is measured from.
 * FNT_E_BUSY: a host-buffer request larger than the whole HBM budget. */
int fnt_session_submit(fnt_session *s, uint32_t ch, const int8_t *in, uint64_t n,
                       int16_t *out, uint32_t flags, uint64_t arrival_ns, uint64_t *ticket);
int fnt_session_poll(fnt_session *s, uint64_t ticket, int *done);
int fnt_session_wait(fnt_session *s, uint64_t ticket);
/* Wait until every submitted request has completed. */
int fnt_session_drain(fnt_session *s);
/* Cancel a request that has not started; FNT_E_STATE if it already runs or ended. */
int fnt_session_cancel(fnt_session *s, uint64_t ticket);
/* Export / import one channel's resident state (taps, overlap tails, stream
 * position) to/from host memory of FNT_STATE_BYTES.  The channel must be idle. */
int fnt_session_get_state(fnt_session *s, uint32_t ch, void *host_buf, size_t *size);
int fnt_session_set_state(fnt_session *s, uint32_t ch, const void *host_buf, size_t size);
int fnt_session_get_stats(fnt_session *s, fnt_session_stats *st);

/* One request of a replayed arrival trace: submitted at start + at_ns. */
typedef struct fnt_request {
    uint32_t ch;
    uint32_t flags;
    const int8_t *in;
    int16_t *out;
    uint64_t n;
    uint64_t at_ns;
} fnt_request;

/* Submit `nreq` requests at their scheduled times (offsets from the call, in
 * ascending order), from the calling thread, with arrival stamped as the
 * scheduled time.  Returns after the last submission; tickets[i] (optional)
 * receive the tickets.  Use fnt_session_drain to wait for completion. */
int fnt_session_replay(fnt_session *s, const fnt_request *reqs, size_t nreq, uint64_t *tickets);
/* Drains outstanding work, then frees everything. */
int fnt_session_destroy(fnt_session *s);

#ifdef __cplusplus
}
#endif

#endif /* FNT_H */
