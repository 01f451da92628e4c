// marfa_level_f32_count.hip -- k_level<float, true, false> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(launch_level_f32_count, float, true, false)
