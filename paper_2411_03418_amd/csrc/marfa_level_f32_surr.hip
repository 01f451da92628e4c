// marfa_level_f32_surr.hip -- k_level<float, false, true> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(launch_level_f32_surr, float, false, true)
