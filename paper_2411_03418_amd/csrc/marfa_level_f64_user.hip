// marfa_level_f64_user.hip -- the level kernel <double, false, false> with the user line shape and chi compiled in, every stencil, and its launcher.
#define MARFA_USER_PLUGINS 1
#define MARFA_STENCILS 7
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f64_user, double, false, false, 1)
