// lc_static.h -- the library's static device scratch (internal).
#pragma once

#include <stddef.h>

// Bytes of the static scratch each GPU holds for allocation-free sweeps.
#define LC_STATIC_SCRATCH_BYTES (64u << 20)

// Device address of the current device's scratch array (set up on first
// use per device), its size in *bytes; nullptr on a HIP error.
void* lc_static_scratch(size_t* bytes);
