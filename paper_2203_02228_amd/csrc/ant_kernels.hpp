// ant_kernels.hpp -- host-side access to the ant kernels, which are compiled
// in their own translation units (one per team size).
#pragma once
#include <hip/hip_runtime.h>

#include "faco_device.hpp"

typedef void (*AntKernelFn)(faco::Inst, int);
typedef void (*AntBatchFn)(const faco::Inst *, const int2 *, int, int, int);
typedef void (*AntPersistFn)(const faco::Inst *, faco::BatchCtl *, faco::BatchRun *, int);

// ant kernel for candidate lists of length k (specialised for KT >= k) with
// tw waves per ant (1, 4 or 8); nullptr for another tw
AntKernelFn faco_ant_kernel(int k, int tw);
// batched ant kernel: one wave per ant (tw = 1, apb ants per workgroup) or
// one workgroup of tw waves per ant (tw = 4, 8)
AntBatchFn faco_ant_batch_kernel(int k, int tw);
// persistent batched ant kernel (all iterations of every instance in one
// launch; one wave per ant, several per workgroup, or tw waves per ant)
AntPersistFn faco_ant_persist_kernel(int k, int tw);
// LDS words of the team area ahead of an ant's bitmaps
int faco_team_lds_words(int tw);
// ant kernel whose local search runs on segment-list tours (Inst.seg_on)
AntKernelFn faco_ant_seg_kernel(int k, int tw);
// LDS words ahead of the segment records of such a kernel (team area and the
// three bitmaps, rounded up to 16 bytes)
int faco_seg_lds_words(int tw, int n);
