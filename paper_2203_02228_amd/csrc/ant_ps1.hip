// ant_ps1.hip -- persistent batched ant kernels with one wave per ant (several per
// workgroup), and the dispatch by team size.
#include "ant_kernels.hpp"
#include "faco_kernels.hpp"

AntPersistFn faco_ant_persist_kernel_tw1(int k) {
  if (k <= 4) return faco::ant_persist_kernel<4, 1>;
  if (k <= 8) return faco::ant_persist_kernel<8, 1>;
  if (k <= 12) return faco::ant_persist_kernel<12, 1>;
  if (k <= 16) return faco::ant_persist_kernel<16, 1>;
  if (k <= 24) return faco::ant_persist_kernel<24, 1>;
  return faco::ant_persist_kernel<32, 1>;
}

AntPersistFn faco_ant_persist_kernel_tw4(int k);
AntPersistFn faco_ant_persist_kernel_tw8(int k);

AntPersistFn faco_ant_persist_kernel(int k, int tw) {
  if (tw == 1) return faco_ant_persist_kernel_tw1(k);
  if (tw == 4) return faco_ant_persist_kernel_tw4(k);
  if (tw == 8) return faco_ant_persist_kernel_tw8(k);
  return nullptr;
}
