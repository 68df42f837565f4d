// ant_sg1.hip -- ant kernels whose local search runs on segment-list tours,
// one wave per ant, and the dispatch by team size.
#include "ant_kernels.hpp"
#include "faco_kernels.hpp"

AntKernelFn faco_ant_seg_kernel_tw1(int k) {
  if (k <= 8) return faco::ant_kernel<8, 1, true>;
  if (k <= 16) return faco::ant_kernel<16, 1, true>;
  return faco::ant_kernel<32, 1, true>;
}

AntKernelFn faco_ant_seg_kernel_tw4(int k);
AntKernelFn faco_ant_seg_kernel_tw8(int k);

AntKernelFn faco_ant_seg_kernel(int k, int tw) {
  if (tw == 1) return faco_ant_seg_kernel_tw1(k);
  if (tw == 4) return faco_ant_seg_kernel_tw4(k);
  if (tw == 8) return faco_ant_seg_kernel_tw8(k);
  return nullptr;
}

int faco_seg_lds_words(int tw, int n) {
  return faco::seg_lds_words(faco_team_lds_words(tw), (n + 31) >> 5);
}
