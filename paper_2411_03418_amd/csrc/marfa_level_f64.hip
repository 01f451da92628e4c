// marfa_level_f64.hip -- the level kernel <double, false, false> without the user line shape and chi, the 3- and 5-point stencils, and its launcher.
#define MARFA_USER_PLUGINS 0
#define MARFA_STENCILS 5
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f64, double, false, false, 1)
