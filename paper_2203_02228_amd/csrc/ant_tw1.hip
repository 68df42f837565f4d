// ant_tw1.hip -- ant kernels with 1 wave(s) per ant.
#include "ant_kernels.hpp"
#include "faco_kernels.hpp"

AntKernelFn faco_ant_kernel_tw1(int k) {
  if (k <= 4) return faco::ant_kernel<4, 1>;
  if (k <= 8) return faco::ant_kernel<8, 1>;
  if (k <= 12) return faco::ant_kernel<12, 1>;
  if (k <= 16) return faco::ant_kernel<16, 1>;
  if (k <= 24) return faco::ant_kernel<24, 1>;
  return faco::ant_kernel<32, 1>;
}

AntBatchFn faco_ant_batch_kernel_tw1(int k) {
  if (k <= 4) return faco::ant_batch_kernel<4, 1>;
  if (k <= 8) return faco::ant_batch_kernel<8, 1>;
  if (k <= 12) return faco::ant_batch_kernel<12, 1>;
  if (k <= 16) return faco::ant_batch_kernel<16, 1>;
  if (k <= 24) return faco::ant_batch_kernel<24, 1>;
  return faco::ant_batch_kernel<32, 1>;
}

AntKernelFn faco_ant_kernel_tw4(int k);
AntKernelFn faco_ant_kernel_tw8(int k);

AntKernelFn faco_ant_kernel(int k, int tw) {
  if (tw == 1) return faco_ant_kernel_tw1(k);
  if (tw == 4) return faco_ant_kernel_tw4(k);
  if (tw == 8) return faco_ant_kernel_tw8(k);
  return nullptr;
}

AntBatchFn faco_ant_batch_kernel_tw4(int k);
AntBatchFn faco_ant_batch_kernel_tw8(int k);

AntBatchFn faco_ant_batch_kernel(int k, int tw) {
  if (tw == 1) return faco_ant_batch_kernel_tw1(k);
  if (tw == 4) return faco_ant_batch_kernel_tw4(k);
  if (tw == 8) return faco_ant_batch_kernel_tw8(k);
  return nullptr;
}

int faco_team_lds_words(int tw) {
  return tw == 1 ? faco::team_words<1>() : faco::team_words<8>();
}
