// ant_sg8.hip -- ant kernels whose local search runs on segment-list tours,
// 8 waves per ant.
#include "ant_kernels.hpp"
#include "faco_kernels.hpp"

AntKernelFn faco_ant_seg_kernel_tw8(int k) {
  if (k <= 8) return faco::ant_kernel<8, 8, true>;
  if (k <= 16) return faco::ant_kernel<16, 8, true>;
  return faco::ant_kernel<32, 8, true>;
}

