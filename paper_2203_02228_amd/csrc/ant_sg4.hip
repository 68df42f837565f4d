// ant_sg4.hip -- ant kernels whose local search runs on segment-list tours,
// 4 waves per ant.
#include "ant_kernels.hpp"
#include "faco_kernels.hpp"

AntKernelFn faco_ant_seg_kernel_tw4(int k) {
  if (k <= 8) return faco::ant_kernel<8, 4, true>;
  if (k <= 16) return faco::ant_kernel<16, 4, true>;
  return faco::ant_kernel<32, 4, true>;
}

