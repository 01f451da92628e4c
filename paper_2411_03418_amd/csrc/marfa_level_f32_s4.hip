// marfa_level_f32_s4.hip -- the level kernel <float, false, false> without the user line shape and chi, the 4-point stencil only, and its launcher.
#define MARFA_USER_PLUGINS 0
#define MARFA_STENCILS 2
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f32_s4, float, false, false, 4)
