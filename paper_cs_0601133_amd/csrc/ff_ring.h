// LDS ring helpers shared by the matrix-core GEMM kernels: operand stages
// are copied global -> LDS by the vector memory unit (global_load_lds) into
// a ring of NST slots, NST - 1 of them in flight while one is consumed.
#pragma once

#include <hip/hip_runtime.h>

namespace ff {

typedef __attribute__((address_space(3))) void *lds_ptr;

// 160 KB of LDS per CU, minus room for small shared variables.
constexpr int LDS_LIMIT = 160 * 1024 - 1024;

// s_waitcnt needs an immediate: wait until at most n vector memory
// operations of this wave are outstanding.
__device__ __forceinline__ void wait_vm(int n)
{
    switch (n) {
#define FF_W(k) case k: asm volatile("s_waitcnt vmcnt(" #k ")" ::: "memory"); break;
        FF_W(0) FF_W(1) FF_W(2) FF_W(3) FF_W(4) FF_W(5) FF_W(6) FF_W(7)
        FF_W(8) FF_W(9) FF_W(10) FF_W(11) FF_W(12) FF_W(13) FF_W(14) FF_W(15)
        FF_W(16) FF_W(17) FF_W(18) FF_W(19) FF_W(20) FF_W(21) FF_W(22) FF_W(23)
        FF_W(24) FF_W(25) FF_W(26) FF_W(27) FF_W(28) FF_W(29) FF_W(30) FF_W(31)
#undef FF_W
    default: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    }
}

// Workgroup barrier without the memory fence of __syncthreads (which would
// make every wave drain all of its outstanding global loads, i.e. every
// stage in flight).  Ordering is explicit instead: each wave waits for its
// own loads of the stage with wait_vm before the barrier, and every read of
// a ring slot feeds a matrix-core instruction issued before the barrier, so
// the slot is free when the barrier completes.  The empty asm statements
// keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void ring_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

} // namespace ff
