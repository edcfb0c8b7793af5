// Error bits that kernels latch in the device control block, and the status
// a call reports for them.  Plain C++ (no HIP): the host runtime and a
// CPU-side unit test both include it; the HIP sources define
// BQS_STATUS_MAP_FN so that kernels can call the mapping too.
#pragma once

#include "bqs.h"

namespace bqs {

enum : unsigned {
    ERR_OVERFLOW = 1u,  // a work list or the level cap ran out of room
    ERR_OFFSETS = 2u,   // malformed segment offsets (nothing else ran)
    ERR_STALL = 4u,     // a bounded device-side wait gave up (look-back or grid barrier)
    ERR_NAN = 8u        // check mode: a floating-point key is NaN
};

// The status of a call whose kernels latched `err`.  Malformed offsets stop
// every kernel, so they win; a NaN found by the check comes next; a stalled
// wait means the device did not run as launched (a HIP-level failure); any
// other bit is a work list that ran out of room.
#ifndef BQS_STATUS_MAP_FN
#define BQS_STATUS_MAP_FN inline
#endif
BQS_STATUS_MAP_FN bqs_status status_of_device_error(unsigned err) {
    if (err == 0) return BQS_OK;
    if (err & ERR_OFFSETS) return BQS_EINVAL;
    if (err & ERR_NAN) return BQS_ENAN;
    if (err & ERR_STALL) return BQS_EHIP;
    return BQS_EOVERFLOW;
}

}  // namespace bqs
