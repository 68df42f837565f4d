// ant_ps4.hip -- persistent batched ant kernels with 4 wave(s) per ant.
#include "ant_kernels.hpp"
#include "faco_kernels.hpp"

AntPersistFn faco_ant_persist_kernel_tw4(int k) {
  if (k <= 4) return faco::ant_persist_kernel<4, 4>;
  if (k <= 8) return faco::ant_persist_kernel<8, 4>;
  if (k <= 12) return faco::ant_persist_kernel<12, 4>;
  if (k <= 16) return faco::ant_persist_kernel<16, 4>;
  if (k <= 24) return faco::ant_persist_kernel<24, 4>;
  return faco::ant_persist_kernel<32, 4>;
}
