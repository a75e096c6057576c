// Small gfx950 device helpers shared by the backprojection and forward
// projection kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdk {

// floor(x) as an integer in one instruction (x is finite and clamped).
__device__ __forceinline__ int cvt_floor(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// a * b + c on 24-bit signed a, b (|a|, |b| < 2^23) in one instruction.
__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// The median of x, lo and hi (x clamped to [lo, hi] when lo <= hi) in one
// instruction.
__device__ __forceinline__ int med3_i32(int x, int lo, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// mad_i24 with a wave-uniform b (read from a scalar register; b must be
// the same in every lane).
__device__ __forceinline__ int mad_i24_ub(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// Raw buffer loads: a 32-bit byte offset per lane, the plane base in a
// buffer descriptor, and the second tap row reached through the scalar
// offset.  An offset outside the descriptor's range would read 0 instead of
// faulting; callers keep every offset inside the buffer.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

// Read-only data that every lane reads at the same address (the folded
// matrices of a batch), seen through the constant address space so that the
// compiler reads it with scalar loads into SGPRs, as it does kernel
// arguments.  The data must not change while the kernel runs.
typedef __attribute__((address_space(4))) const float const_float;
__device__ __forceinline__ const const_float* as_constant(const float* p)
{
    return (const const_float*)p;
}

}  // namespace fdk
