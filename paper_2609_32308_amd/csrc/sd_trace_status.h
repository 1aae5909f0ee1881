// Status codes of the device traceback, shared by the trace kernels and the host check.
#pragma once

namespace sd {

// Status the device traceback reports (TraceOut::status).
enum TraceStatus : int {
    kTrOk = 1,
    kTrNoMatch = 2,      // a decision found no alternative equal to its stored value
    kTrDup = 3,          // a position was emitted twice
    kTrWait = 4,         // a wait for the frame stack exceeded its spin limit
    kTrFrame = 5,        // a deferred frame named states outside the design
    kTrStack = 6,        // more deferred frames than the stack holds
    kTrUnreachable = 7,  // X(s) is infinite
};

}  // namespace sd
