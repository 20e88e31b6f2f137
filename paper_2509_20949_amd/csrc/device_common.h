// device_common.h -- small device helpers shared by the BCC and FCC sweep
// kernels.
#pragma once

#include "smcx_internal.h"

namespace smcx {

// Species codes in LDS: species v is stored as (F + 32) * v, F the width of
// its histogram field; the top 3 bits give v back.
__device__ __forceinline__ uint32_t decode(uint32_t code) { return code >> 5; }

// acc + a * b on the 24-bit multiplier (a, b signed 24-bit), modulo 2^32
__device__ __forceinline__ uint32_t mad24(uint32_t a, int32_t b, uint32_t acc)
{
    return (uint32_t)__mul24((int32_t)a, b) + acc;
}

// Cell (3 ix, 3 iy, 3 iz) of a 4 x 4 x 4 sub-colour round taken by `lane`:
// lane bits 0 and 5 give ix, bits 1-2 iy, bits 3-4 iz.  Each half-wave then
// covers two x columns, which with the 231-byte plane pitch puts its 32 byte
// reads at any common offset into distinct LDS banks.
__device__ __forceinline__ void lane_cell(int lane, int& ix, int& iy, int& iz)
{
    ix = (lane & 1) | ((lane >> 4) & 2);
    iy = (lane >> 1) & 3;
    iz = (lane >> 3) & 3;
}

__device__ __forceinline__ int wrap_add(int v, int L)   // v in [-L, 2L)
{
    v = v < 0 ? v + L : v;
    return v >= L ? v - L : v;
}

}  // namespace smcx
