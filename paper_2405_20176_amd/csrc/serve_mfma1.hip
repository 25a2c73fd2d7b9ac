// Instantiations of the matrix-core alert kernel for d in {9, ..., 16}.
#include "serve_mfma.cuh"

namespace snaps {

AlertKernel alert_mfma_pick_group1(int D, int kc) {
    switch (D) {
        case 9: return alert_mfma_kc<9>(kc);
        case 10: return alert_mfma_kc<10>(kc);
        case 11: return alert_mfma_kc<11>(kc);
        case 12: return alert_mfma_kc<12>(kc);
        case 13: return alert_mfma_kc<13>(kc);
        case 14: return alert_mfma_kc<14>(kc);
        case 15: return alert_mfma_kc<15>(kc);
        case 16: return alert_mfma_kc<16>(kc);
    }
    return nullptr;
}

}  // namespace snaps
