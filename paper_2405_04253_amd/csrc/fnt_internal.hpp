// Internal interfaces between the C-ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fnt.h"

namespace fnti {

// One channel's CDC work: 32 new instants per overlap-save block.
struct CdcItem {
    const int8_t *in;      // [n][4]
    const int8_t *hist;    // [32][4] instants preceding in[0], or nullptr (zeros)
    int32_t *z_out;        // [n][4] or nullptr
    int8_t *a_out;         // [M][4] or nullptr, M = (n + 1 - phase) / 2
    uint64_t n;
    uint64_t block0;       // first global block index of this item (prefix sum)
    uint64_t chunk0;       // first global chunk (CDC_CHUNK blocks of this item) index (prefix sum)
    int8_t taps[32][2];
    int32_t ntaps;
    int32_t shift;
    int32_t phase;
    int32_t pad_;
};

// The lane-per-block CDC kernel gives each wave one chunk: up to CDC_CHUNK
// consecutive blocks of one item, one block per lane.
constexpr int CDC_CHUNK = 64;

// One channel's AEQ run over m symbols (serial chain of 16-symbol blocks).
struct AeqItem {
    const int8_t *a;       // [m][4]
    int16_t *out;          // [m][4]
    int16_t *taps;         // [4][4][16] in/out
    const int8_t *hist_in; // [16][4] symbols preceding a[0], or nullptr (zeros)
    int8_t *hist_out;      // [16][4] receives the last 16 symbols, or nullptr
    const int8_t *cdc_in;  // CDC input of this run, for the CDC tail update
    int8_t *cdc_tail;      // [32][4] CDC history (in/out), or nullptr: no update
    uint64_t cdc_n;        // instants in cdc_in
    uint64_t m;
    int32_t out_shift;
    int32_t err_shift;
    int32_t mu_shift;
    int32_t const_unit;
    int32_t update_enable;
    int32_t mu_shift_late;     // step schedule: blocks block0 + b >= gear_blocks (> 0) use mu_shift_late
    uint32_t gear_blocks;
    uint32_t pad_;
    uint64_t block0;           // stream index of this run's first block (sessions: the stream position)
};

__host__ __device__ inline uint64_t cdc_blocks(uint64_t n) { return (n + 31) / 32; }
__host__ __device__ inline uint64_t cdc_chunks(uint64_t n) { return (cdc_blocks(n) + CDC_CHUNK - 1) / CDC_CHUNK; }
__host__ __device__ inline uint64_t n_symbols(uint64_t n, int phase) {
    return n + 1 > (uint64_t)phase ? (n + 1 - (uint64_t)phase) / 2 : 0;
}

// Bit of the per-device error flag latched when a bounded wait of the fused
// kernel gave up (the other bits are range violations).
constexpr int kFlagStall = 16;
// Bit latched when a channel descriptor read on the device was invalid.
constexpr int kFlagParam = 32;
// Polls a fused-kernel wait makes before it gives up (seconds of waiting).
constexpr uint32_t kFusedSpinLimit = 1u << 22;

// Launchers (fnt_kernels.hip).  `items` is a device table or nullptr, in which
// case `single` is used (passed by value in the kernel arguments).
hipError_t launch_transform(const uint32_t *x, uint32_t *X, size_t batch, int t, int log2n,
                            int alpha_kind, bool inverse, int *err, hipStream_t s);
// CDC variant 0 (default): one block per lane, CDC_CHUNK blocks per wave, the
// 64-point transforms in registers; needs total_chunks (sum of cdc_chunks) and
// waves_per_group; blocks_per_wave is unused.  Variant 1: one block per wave,
// 16 lanes per transform, blocks_per_wave consecutive blocks per wave.  The
// exact output z (with_z) always takes variant 1.  Variant 2: the direct
// time-domain comparator (no Fermat-domain arithmetic), chunks as variant 0.
hipError_t launch_cdc(const CdcItem *items, int nitems, const CdcItem &single,
                      uint64_t total_blocks, uint64_t total_chunks, int variant,
                      int waves_per_group, int blocks_per_wave, bool with_z, int *err,
                      hipStream_t s);
// One launch for the split of a longest-first table: items [0, nlong) in form
// form_long at raised wave priority (dispatched first), the rest in form_rest
// (at raised priority too with rest_high_priority).
// Fusable pairs: long form 1, 2, 4 or 5 with rest 0 or 3, (3, 0) and (2, 5).
hipError_t launch_aeq_split(const AeqItem *items, int nlong, int nitems, int form_long, int form_rest,
                           int *err, hipStream_t s, bool rest_high_priority = false);
bool aeq_split_fusable(int form_long, int form_rest);
// variant 0: Fermat-domain AEQ in form waves_per_pol (0 lane, 3 duo, 1 / 2 / 4
// split by output polarisation with that many waves per half, 5 split by output
// polarisation with both halves in one workgroup); 1: direct time-domain
// comparator; 2: Fermat-domain, one wave per channel.
// Fused persistent CDC + AEQ in one launch (cdc_aeq_fused_kernel), AEQ in the
// polarisation-split form with lpt lanes per transform (4, 8 or 16: one, two or
// four waves per half) and one CDC producer wave per workgroup.  Tables
// citems / aitems: the same channels in the same order (longest chains first),
// aitems[i].m = n_symbols(citems[i].n, phase); or both nullptr and the single
// items cs / as.  With queue (two device words, zero before the first launch;
// every launch leaves them zero) grid <= channels workgroups take channels in
// table order; without, grid = channels and workgroup w runs channel w.
// Channels [0, nprio) run at raised wave priority.  split_halves: one
// workgroup per polarisation half, each computing the CDC itself (for idle
// GPUs: the halves' waves get a CU each), grid = fused_split_grid(channels),
// no queue.
hipError_t launch_fused(const CdcItem *citems, const AeqItem *aitems, int n, const CdcItem &cs,
                        const AeqItem &as, int lpt, uint32_t *queue, unsigned grid, int nprio, int *err,
                        hipStream_t s, bool split_halves = false, uint32_t spin_limit = kFusedSpinLimit);
unsigned fused_split_grid(int n);
// Workgroups of the fused kernel resident at once on the current device (0 on error).
int fused_capacity(int lpt);
hipError_t launch_aeq(const AeqItem *items, int nitems, const AeqItem &single, int variant,
                      int waves_per_pol, int *err, hipStream_t s,
                      bool high_priority = false);

}  // namespace fnti
