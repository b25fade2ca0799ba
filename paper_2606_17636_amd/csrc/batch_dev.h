// Device side of the batched launch lists (BatchRef in smg_internal.h).
#pragma once
#include <hip/hip_runtime.h>

#include "smg_internal.h"

// Resolve list position p of a launch: false for a block beyond the device
// list length.  The count and the entry are read by two independent loads
// that the exit test needs both of, so they are in flight together (a test
// on the count alone would let the compiler issue the entry's load only
// after the count has arrived).  The list holds cap >= 1 entries, so p is
// always in range, and the first entry stands in for the count's address
// when the list has no device length.  Entries are non-negative.
__device__ __forceinline__ bool batch_entry(const BatchRef& bt, int p, int& e) {
  const int* const cptr = bt.count ? bt.count : bt.ent;
  const int craw = *cptr;
  e = bt.ent[p];
  const int cnt = bt.count ? craw : bt.cap;
  return p < cnt && e >= 0;
}

// Holds a uniform value in scalar registers at this point of the program:
// the loads that produce the values pinned together are issued before it
// and waited for once, instead of each being issued where it is first used
// (past branches that would otherwise wait for earlier loads one by one).
__device__ __forceinline__ void pin_scalar(int v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void pin_scalar(const void* v) { asm volatile("" ::"s"(v)); }
