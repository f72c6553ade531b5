// Chain-step launches for factors stored in FP64 (kernels in chain_kernels.h).
#include "chain_kernels.h"

void chain_launch_f64(const IterArgs& a, hipStream_t st) { chain_launch_vt<double>(a, st); }

void spmv_halo_launch(const IterArgs& a, int par, hipStream_t st) {
  MORX_NC_DISPATCH(a.ncv_spmv, spmv_halo_run<NC>(a, par, st));
}
