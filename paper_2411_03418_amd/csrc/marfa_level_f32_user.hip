// marfa_level_f32_user.hip -- the level kernel <float, false, false> with the user line shape and chi compiled in, every stencil, and its launcher.
#define MARFA_USER_PLUGINS 1
#define MARFA_STENCILS 7
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f32_user, float, false, false, 4)
