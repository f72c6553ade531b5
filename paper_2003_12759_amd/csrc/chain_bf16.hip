// Chain-step launches for factors stored in BF16 (kernels in chain_kernels.h).
#include "chain_kernels.h"

void chain_launch_bf16(const IterArgs& a, hipStream_t st) { chain_launch_vt<uint16_t>(a, st); }
