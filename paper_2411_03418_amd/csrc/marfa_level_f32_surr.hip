// marfa_level_f32_surr.hip -- the level kernel <float, false, true> without the user line shape and chi, the 3-point stencil, and its launcher.
#define MARFA_USER_PLUGINS 0
#define MARFA_STENCILS 1
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f32_surr, float, false, true, 3)
