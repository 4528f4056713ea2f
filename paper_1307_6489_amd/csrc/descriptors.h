// Checks of the ragged batch descriptors, shared by the fused reconstruction
// kernel and the per-array-event kernel.  Plain C++ apart from the
// __host__ __device__ qualifiers, so a host driver compiled with g++ (the
// qualifiers defined empty) runs exactly these functions.
//
// A batch is a pool of uint16 trace elements, one (type, offset) descriptor
// per camera event, and per array event a range [lo, hi) of camera events
// (the event builder's merged array event).  Descriptors come from outside the
// library; a rejected one only sets a status bit and a record flag.
#pragma once

#include <cstdint>

#include "rta.h"

namespace rta {

// Status bits of one camera-event descriptor: RTA_STATUS_BAD_TYPE if the type
// index is outside [0, n_types) (elems_of is then not called), else
// RTA_STATUS_BAD_OFFSET if the offset is negative, is not a multiple of 8
// elements (the 16-byte alignment of the vector trace loads), or the event's
// elems_of(type) elements do not fit in the pool of pool_len elements; 0 for
// a valid descriptor, whose event is then the elements [off, off + elems) of
// the pool.  Written without sums that could overflow for any int64 offset.
template <class ElemsOf>
__host__ __device__ inline uint32_t tel_descriptor_status(int32_t ty, int64_t off, int32_t n_types, int64_t pool_len,
                                                          ElemsOf elems_of) {
  if (ty < 0 || ty >= n_types) return RTA_STATUS_BAD_TYPE;
  const int64_t n = elems_of(ty);
  if (off < 0 || (off & 7) != 0 || n < 0 || n > pool_len || off > pool_len - n) return RTA_STATUS_BAD_OFFSET;
  return 0u;
}

// An array event's camera-event range [lo, hi) is usable iff it lies inside
// the batch's n_tel camera events (an empty range is valid).
__host__ __device__ inline bool event_range_ok(int64_t lo, int64_t hi, int64_t n_tel) {
  return lo >= 0 && lo <= hi && hi <= n_tel;
}

}  // namespace rta
