// Stand-in for the HIP runtime header in the host emulation build.
#pragma once
#include "../../hip_emu.h"
