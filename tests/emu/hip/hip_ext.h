// CPU emulation of hipExtLaunchKernelGGL (test infrastructure only): the
// launch runs like any other; the timing events are ignored.
#pragma once
#include "hip_runtime.h"
#define hipExtLaunchKernelGGL(K, G, B, S, STREAM, E0, E1, FL, ...) \
  emu_launch(K, dim3(G), dim3(B), (size_t)(S), __VA_ARGS__)
