// Device helpers shared by the libsnaps kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace snaps {

// Pointers into read-only memory that every lane of a wavefront reads at the
// same address.  Address space 4 (constant) tells the compiler the data is
// invariant for the kernel's lifetime, so uniform reads become scalar loads
// into SGPRs that every lane then uses as an operand.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)(p);
}

// v_writelane_b32: lane `lane` of the result takes `val` (wavefront-uniform),
// every other lane keeps `old`.
__device__ int lane_write(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// Waits written as asm with a memory clobber, so that the compiler neither
// moves memory accesses across them nor keeps LDS values in registers
// across them: at most N vector memory operations of this wavefront still
// outstanding (global-to-LDS copies included, which the compiler does not
// track), and all LDS operations complete.
template <int N>
__device__ __forceinline__ void wait_vmem() {
    static_assert(N >= 0 && N < 16, "vmcnt field");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
__device__ __forceinline__ void wait_lds() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Minimum / maximum over each 32-lane half of the wavefront.
__device__ __forceinline__ float half_min(float v) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float half_max(float v) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// h[bin] += 1 for every lane of the wavefront with active set, with one LDS
// atomic per distinct bin (lanes of one bin are counted by a ballot): keys
// that crowd into few bins (small integer counts) would otherwise serialise
// on one address.  Must be called by every lane of the wavefront.
__device__ __forceinline__ void wave_hist_add(unsigned* h, uint32_t bin, bool active) {
    const int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(active);
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)bin, leader);
        const bool mine = ((pending >> lane) & 1ull) != 0ull;
        const unsigned long long same = __ballot(mine && bin == b);
        if (lane == leader) atomicAdd(&h[b], (unsigned)__popcll(same));
        pending &= ~same;
    }
}

// Inclusive scan over a 64-lane wavefront.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

// Inclusive scan over a 64-lane wavefront with DPP row shifts and row
// broadcasts (no LDS traffic): shifts by 1, 2, 4 and 8 within each row of 16
// lanes, then row 0's last lane into row 1 (and row 2's into row 3), then
// lane 31 into rows 2 and 3.  Lanes with no source add 0.
__device__ __forceinline__ int wave_scan_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return v;
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_move_f64(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, kCtrl, kRowMask, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), kCtrl, kRowMask, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The same scan on doubles (both halves moved by DPP); lane 63 ends with
// the sum over the wavefront.
__device__ __forceinline__ double wave_scan_dpp(double v) {
    v += dpp_move_f64<0x111, 0xf>(v);
    v += dpp_move_f64<0x112, 0xf>(v);
    v += dpp_move_f64<0x114, 0xf>(v);
    v += dpp_move_f64<0x118, 0xf>(v);
    v += dpp_move_f64<0x142, 0xa>(v);
    v += dpp_move_f64<0x143, 0xc>(v);
    return v;
}

// Exclusive scan over the whole workgroup (blockDim.x a multiple of 64,
// at most 1024).  tmp needs 17 ints of LDS.  Returns the exclusive prefix
// and writes the workgroup total to *total.  Contains three barriers, so
// consecutive calls may reuse tmp.
__device__ __forceinline__ int block_exclusive_scan(int v, int* tmp, int* total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int inc = wave_inclusive_scan(v);
    if (lane == 63) tmp[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        int w = lane < nw ? tmp[lane] : 0;
        int wi = wave_inclusive_scan(w);
        if (lane < nw) tmp[lane] = wi - w;
        if (lane == nw - 1) tmp[16] = wi;
    }
    __syncthreads();
    const int tot = tmp[16];
    const int base = tmp[wave];
    __syncthreads();
    *total = tot;
    return inc - v + base;
}

// Ascending bitonic sort of P (a power of two) unsigned keys in LDS by the
// whole workgroup.  Ends with a barrier.
template <typename K>
__device__ __forceinline__ void bitonic_sort_lds(K* buf, int P) {
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = threadIdx.x; p < (P >> 1); p += blockDim.x) {
                const int i = 2 * p - (p & (j - 1));
                const int l = i + j;
                const K a = buf[i];
                const K b = buf[l];
                const bool up = (i & k) == 0;
                if ((a > b) == up) {
                    buf[i] = b;
                    buf[l] = a;
                }
            }
            __syncthreads();
        }
    }
}

__host__ __device__ inline int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace snaps
