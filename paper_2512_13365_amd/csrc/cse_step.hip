// cse_step.hip -- the step kernels of one row-word count, CSE_STEP_W (1..8,
// set by the build), and the lookup of a class's kernel (cse_step.hpp).
#define CSE_STEP_TU 1
#include "cse_kernels.hpp"
#include "cse_step.hpp"

#ifndef CSE_STEP_W
#error "CSE_STEP_W (row words, 1..8) must be defined"
#endif

namespace {

template <bool GS, bool ADJ, bool TL>
const void* kernel_nw(int nw) {
    constexpr int W = CSE_STEP_W;
    if constexpr (ADJ) {
        switch (nw) {
        case 1: return (const void*)csek::step_kernel<W, GS, ADJ, TL, 1>;
        case 2: return (const void*)csek::step_kernel<W, GS, ADJ, TL, 2>;
        case 4: return (const void*)csek::step_kernel<W, GS, ADJ, TL, 4>;
        default: return nullptr;
        }
    } else {
        return nw == 1 ? (const void*)csek::step_kernel<W, GS, ADJ, TL, 1> : nullptr;
    }
}

const void* kernel_of(bool gs, bool adj, bool tl, int nw) {
    if (gs && adj) return tl ? kernel_nw<true, true, true>(nw) : kernel_nw<true, true, false>(nw);
    if (tl) return nullptr;
    if (gs) return kernel_nw<true, false, false>(nw);
    return adj ? kernel_nw<false, true, false>(nw) : kernel_nw<false, false, false>(nw);
}

}  // namespace

#define CSE_STEP_NAME2(w) csek_step_kernel_w##w
#define CSE_STEP_NAME(w) CSE_STEP_NAME2(w)

extern "C" const void* CSE_STEP_NAME(CSE_STEP_W)(bool gs, bool adj, bool tl, int nw) {
    return kernel_of(gs, adj, tl, nw);
}
