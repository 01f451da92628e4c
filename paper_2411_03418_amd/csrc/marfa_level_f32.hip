// marfa_level_f32.hip -- the level kernel <float, false, false> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f32, float, false, false, 4)
