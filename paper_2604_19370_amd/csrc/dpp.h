// dpp.h -- cross-lane moves of a 64-lane wavefront through DPP (data-parallel
// primitives: the operand is routed between lanes inside the VALU, no LDS
// crossbar).  Lane layouts on gfx950:
//   wave_rol1: lane i <- lane (i+1) mod 64      wave_shr1: lane i <- lane i-1 (lane 0 keeps `old`)
//   row_shr n: lane i <- lane i-n within rows of 16 (lanes below n in the row keep `old`)
//   row_bcast15: lanes of row r>0 <- lane 16r-1;  row_bcast31: lanes 32..63 <- lane 31
#pragma once
#include <hip/hip_runtime.h>

namespace iga {

enum : int {
    DPP_ROW_SHR1 = 0x111,
    DPP_ROW_SHR2 = 0x112,
    DPP_ROW_SHR4 = 0x114,
    DPP_ROW_SHR8 = 0x118,
    DPP_WAVE_ROL1 = 0x134,
    DPP_WAVE_SHR1 = 0x138,
    DPP_ROW_BCAST15 = 0x142,
    DPP_ROW_BCAST31 = 0x143,
};

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float old, float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL,
                                                      ROW_MASK, 0xf, false));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp(double old, double x)
{
    const long long o = __double_as_longlong(old), v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)v, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, ROW_MASK,
                                               0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP move with every lane written (no `old` operand): invalid source lanes
// read zero
template <int CTRL> __device__ __forceinline__ float dpp_mov(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL> __device__ __forceinline__ double dpp_mov(double x)
{
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// value of lane i+B (B >= 1): lanes 64-B .. 63 receive `halo` of lanes 0 .. B-1
template <int B, typename T> __device__ __forceinline__ T lane_ahead(T x, T halo, int lane)
{
    T v = lane < B ? halo : x;
#pragma unroll
    for (int k = 0; k < B; ++k) v = dpp_mov<DPP_WAVE_ROL1>(v);
    return v;
}

// value of lane i-B (B >= 1); lanes below B receive zero
template <int B, typename T> __device__ __forceinline__ T lane_behind(T x)
{
#pragma unroll
    for (int k = 0; k < B; ++k) x = dpp_mov<DPP_WAVE_SHR1>(x);
    return x;
}

}  // namespace iga
