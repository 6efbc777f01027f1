// cse_step.hpp -- the step kernels of each row-word count W live in their
// own translation unit (cse_step.hip compiled once per W), so the classes
// compile in parallel.  csek_step_kernel_wW returns the host handle of the
// kernel step_kernel<W, gs, adj, tl, nw> for hipLaunchKernel and
// hipFuncSetAttribute, or null when that class does not exist (tl without
// gs and adj; nw other than 1, 2, 4; nw > 1 without adj).
#pragma once

extern "C" {
const void* csek_step_kernel_w1(bool gs, bool adj, bool tl, int nw);
const void* csek_step_kernel_w2(bool gs, bool adj, bool tl, int nw);
const void* csek_step_kernel_w3(bool gs, bool adj, bool tl, int nw);
const void* csek_step_kernel_w4(bool gs, bool adj, bool tl, int nw);
const void* csek_step_kernel_w5(bool gs, bool adj, bool tl, int nw);
const void* csek_step_kernel_w6(bool gs, bool adj, bool tl, int nw);
const void* csek_step_kernel_w7(bool gs, bool adj, bool tl, int nw);
const void* csek_step_kernel_w8(bool gs, bool adj, bool tl, int nw);
}
