// Instantiations of the matrix-core join kernel for d in {9, ..., 16}, the leaner walk (H = 0).
#include "join_mfma.cuh"

namespace snaps {

JoinFn join_mfma_pick_group1(int D, int kc) {
    switch (D) {
        case 9: return join_mfma_pick_kc<9, 0>(kc);
        case 10: return join_mfma_pick_kc<10, 0>(kc);
        case 11: return join_mfma_pick_kc<11, 0>(kc);
        case 12: return join_mfma_pick_kc<12, 0>(kc);
        case 13: return join_mfma_pick_kc<13, 0>(kc);
        case 14: return join_mfma_pick_kc<14, 0>(kc);
        case 15: return join_mfma_pick_kc<15, 0>(kc);
        case 16: return join_mfma_pick_kc<16, 0>(kc);
    }
    return nullptr;
}

}  // namespace snaps
