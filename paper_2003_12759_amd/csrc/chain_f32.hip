// Chain-step launches for factors stored in FP32 (kernels in chain_kernels.h).
#include "chain_kernels.h"

void chain_launch_f32(const IterArgs& a, hipStream_t st) { chain_launch_vt<float>(a, st); }
