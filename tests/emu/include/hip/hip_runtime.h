// Stand-in for the HIP runtime header in the CPU emulation build of the
// device code (tests/emu): device sources include <hip/hip_runtime.h>, and
// the emulation's include directory comes first on the search path.
#pragma once
#include "../../hip_emu.h"
