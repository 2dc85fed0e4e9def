// Stand-in for <hip/hip_ext.h> in the host emulation: hipExtLaunchKernelGGL
// is defined by the emulated hip_runtime.h.
#pragma once
#include "hip_runtime.h"
