// marfa_level_f64_count.hip -- the level kernel <double, true, false> without the user line shape and chi, every stencil, and its launcher.
#define MARFA_USER_PLUGINS 0
#define MARFA_STENCILS 7
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f64_count, double, true, false, 1)
