// Host helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fnt_internal.hpp"

namespace fnti {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int device_err_flag(int **out);
int validate_cdc(const fnt_cdc_params *p);
int validate_aeq(const fnt_aeq_params *p);
bool aligned(const void *p, size_t a);
void fill_cdc_item(CdcItem &it, const int8_t *in, uint64_t n, const fnt_cdc_params *p);
void fill_aeq_item(AeqItem &it, const int8_t *a, uint64_t m, int16_t *taps, const fnt_aeq_params *p,
                   int16_t *out);
void default_cdc_schedule(uint64_t total_blocks, int *wpg, int *bpw);
hipError_t run_cdc(const CdcItem *items, int nitems, const CdcItem &single, uint64_t blocks,
                   uint64_t chunks, int wpg, int bpw, bool with_z, int *err, hipStream_t s);

}  // namespace fnti
