// marfa_level_f32_surr.hip -- the level kernel <float, false, true> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f32_surr, float, false, true, 3)
