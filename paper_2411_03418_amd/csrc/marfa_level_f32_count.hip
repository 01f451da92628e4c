// marfa_level_f32_count.hip -- the level kernel <float, true, false> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f32_count, float, true, false, 1)
