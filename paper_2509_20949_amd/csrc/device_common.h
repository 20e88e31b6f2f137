// device_common.h -- small device helpers shared by the BCC and FCC sweep
// kernels.
#pragma once

#include "smcx_internal.h"

namespace smcx {

// Species codes in LDS: species v is stored as (F + 32) * v, F the width of
// its histogram field; the top 3 bits give v back.
__device__ __forceinline__ uint32_t decode(uint32_t code) { return code >> 5; }

// acc + a * b on the 24-bit multiplier (a, b signed 24-bit), modulo 2^32:
// one v_mad_i32_i24 (the compiler otherwise splits it into a multiply and a
// three-input add)
__device__ __forceinline__ uint32_t mad24(uint32_t a, int32_t b, uint32_t acc)
{
    uint32_t r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(acc));
    return r;
}

__device__ __forceinline__ int wrap_add(int v, int L)   // v in [-L, 2L)
{
    v = v < 0 ? v + L : v;
    return v >= L ? v - L : v;
}

}  // namespace smcx
