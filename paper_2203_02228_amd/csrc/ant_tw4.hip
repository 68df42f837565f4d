// ant_tw4.hip -- ant kernels with 4 wave(s) per ant.
#include "ant_kernels.hpp"
#include "faco_kernels.hpp"

AntKernelFn faco_ant_kernel_tw4(int k) {
  if (k <= 4) return faco::ant_kernel<4, 4>;
  if (k <= 8) return faco::ant_kernel<8, 4>;
  if (k <= 12) return faco::ant_kernel<12, 4>;
  if (k <= 16) return faco::ant_kernel<16, 4>;
  if (k <= 24) return faco::ant_kernel<24, 4>;
  return faco::ant_kernel<32, 4>;
}

AntBatchFn faco_ant_batch_kernel_tw4(int k) {
  if (k <= 4) return faco::ant_batch_kernel<4, 4>;
  if (k <= 8) return faco::ant_batch_kernel<8, 4>;
  if (k <= 12) return faco::ant_batch_kernel<12, 4>;
  if (k <= 16) return faco::ant_batch_kernel<16, 4>;
  if (k <= 24) return faco::ant_batch_kernel<24, 4>;
  return faco::ant_batch_kernel<32, 4>;
}
