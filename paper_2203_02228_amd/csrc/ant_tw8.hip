// ant_tw8.hip -- ant kernels with 8 wave(s) per ant.
#include "ant_kernels.hpp"
#include "faco_kernels.hpp"

AntKernelFn faco_ant_kernel_tw8(int k) {
  if (k <= 4) return faco::ant_kernel<4, 8>;
  if (k <= 8) return faco::ant_kernel<8, 8>;
  if (k <= 12) return faco::ant_kernel<12, 8>;
  if (k <= 16) return faco::ant_kernel<16, 8>;
  if (k <= 24) return faco::ant_kernel<24, 8>;
  return faco::ant_kernel<32, 8>;
}

AntBatchFn faco_ant_batch_kernel_tw8(int k) {
  if (k <= 4) return faco::ant_batch_kernel<4, 8>;
  if (k <= 8) return faco::ant_batch_kernel<8, 8>;
  if (k <= 12) return faco::ant_batch_kernel<12, 8>;
  if (k <= 16) return faco::ant_batch_kernel<16, 8>;
  if (k <= 24) return faco::ant_batch_kernel<24, 8>;
  return faco::ant_batch_kernel<32, 8>;
}
