// Stand-in for <hip/hip_runtime.h> when the device headers are compiled as
// host C++ by the CPU emulation (tests/emu).
#pragma once
#include "../hip_emu.h"
