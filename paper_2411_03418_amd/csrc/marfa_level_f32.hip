// marfa_level_f32.hip -- k_level<float, false, false> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(launch_level_f32, float, false, false)
