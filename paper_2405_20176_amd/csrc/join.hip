// Dispatch of the fused join kernel over its instantiations (dimensionality,
// top-k capacity, prefilter flavour), occupancy query and launch.
#include "join_kernel.cuh"
#include "join_mfma.cuh"

namespace snaps {

int kc_class(int k) {
    if (k <= 0) return 0;
    if (k <= 5) return 5;
    if (k <= 10) return 10;
    if (k <= 20) return 20;
    return 32;
}

size_t join_lds_bytes(int kc, int split) {
    if (split <= 1) return 0;   // also the matrix-core kernel (always one wavefront)
    const int ks = kc > 0 ? kc : 1;
    // per wavefront and query slot: top-k list keys, eps counts, then
    // the float64 eps sums (the offset of the last block is a multiple of 256)
    return (size_t)split * join_ql(kc) * (ks * 64 * 8 + 64 * 4 + 64 * 8);
}

namespace {

// xf: 0 direct form, 1 vector-ALU prefilter, 2 matrix-core prefilter;
// hier: the matrix-core kernel's walk with super-tile and candidate-half
// culls (the vector-ALU kernels have one walk).
JoinFn pick(int D, int kc, int xf, int hier) {
    if (xf == 2) {
        if (D >= 2 && D <= 8) return hier ? join_mfma_pick_group2(D, kc) : join_mfma_pick_group0(D, kc);
        if (D >= 9 && D <= 16) return hier ? join_mfma_pick_group3(D, kc) : join_mfma_pick_group1(D, kc);
        return nullptr;
    }
    if (D >= 2 && D <= 6) return join_pick_group0(D, kc, xf);
    if (D >= 7 && D <= 10) return join_pick_group1(D, kc, xf);
    if (D >= 11 && D <= 13) return join_pick_group2(D, kc, xf);
    if (D >= 14 && D <= 16) return join_pick_group3(D, kc, xf);
    return nullptr;
}

}  // namespace

int join_blocks_per_cu(int D, int kc, int xf, int hier, int split, int mq) {
    JoinFn fn = pick(D, kc, xf, hier);
    if (!fn) return 0;
    int nb = 0;
    const int threads = 64 * (split > mq ? split : mq);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn), threads,
                                                     join_lds_bytes(kc, split)) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_join(int D, int kc, int xf, int hier, const JoinArgs& a, int grid, hipStream_t s) {
    JoinFn fn = pick(D, kc, xf, hier);
    if (!fn) return hipErrorInvalidValue;
    JoinArgs copy = a;
    void* args[] = {&copy};
    const int threads = 64 * (a.split > a.mq ? a.split : a.mq);
    return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(grid), dim3(threads), args,
                           join_lds_bytes(kc, a.split), s);
}

}  // namespace snaps
