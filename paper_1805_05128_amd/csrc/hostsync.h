// Small results handed to the host through pinned memory that the host polls (k_bin.hip):
// the mesh bounds, and single device words (the CFL step's minimum), instead of a
// device-to-host copy and a stream synchronisation.
#pragma once

#include "csph_internal.h"

namespace csph {

// Fine-grained (coherent) host memory the bounds kernel writes: min x, y, z, max x, y, z,
// max d, then the call's sequence number, stored last with a system-scope release.
struct alignas(64) HostBounds {
    double b[8];
    unsigned long long seq;
};

// launch_bounds, whose final reduction also writes the seven values and then `seq` to hb.
hipError_t launch_bounds_host(const double *x, const double *y, const double *z,
                              const double *d, int64_t n, double *part, double *out,
                              HostBounds *hb, unsigned long long seq, hipStream_t st);

// One 64-bit word to the slot (as b[0]'s bits), then `seq`, as launch_bounds_host does.
hipError_t launch_word_host(const unsigned long long *src, HostBounds *hb,
                            unsigned long long seq, hipStream_t st);

}  // namespace csph
