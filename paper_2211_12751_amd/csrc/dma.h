// Direct (DMA) loads from global memory into LDS for the tile rings of the query pass.
//
// buffer_load_dword{,x4} ... lds writes each lane's 4 (16) bytes at M0 + 4 (16) x lane,
// read through a raw buffer descriptor: bytes at or past num_records read as zero.  The
// loads are written as asm blocks with no register outputs, so the compiler neither
// counts them nor orders later LDS reads behind them: a kernel that issues them waits
// for them itself (vmcnt, whose count covers every earlier VMEM operation of the wave,
// as they complete in order), then crosses a barrier before any wave reads the data.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rk {

typedef unsigned int dma_rsrc __attribute__((ext_vector_type(4)));

// raw buffer descriptor of [base, base + bytes), stride 0
__device__ __forceinline__ dma_rsrc dma_buffer(const void* base, uint32_t bytes)
{
    const uint64_t b = (uint64_t)base;
    dma_rsrc r;
    r.x = (uint32_t)b;
    r.y = (uint32_t)(b >> 32) & 0xffffu;
    r.z = bytes;
    r.w = 0x00020000u;
    return r;
}
__device__ __forceinline__ void dma_load16(dma_rsrc rsrc, uint32_t lds, uint32_t voff)
{
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
                 :
                 : "s"(lds), "v"(voff), "s"(rsrc)
                 : "memory", "m0");
}
__device__ __forceinline__ void dma_load4(dma_rsrc rsrc, uint32_t lds, uint32_t voff)
{
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dword %1, %2, 0 offen lds"
                 :
                 : "s"(lds), "v"(voff), "s"(rsrc)
                 : "memory", "m0");
}
// LDS byte address of a __shared__ object (the M0 operand above)
#define RK_LDS_ADDR(p) ((uint32_t)(uintptr_t)((__attribute__((address_space(3))) void*)(p)))

// wait until at most n VMEM operations of this wave are outstanding (n < 64; lgkm and
// export counts left at their maxima)
#define RK_WAIT_VMCNT(n) __builtin_amdgcn_s_waitcnt(((n) & 15) | (((n) >> 4) << 14) | (7 << 4) | (15 << 8))

}  // namespace rk
