// marfa_level_f32.hip -- the level kernel <float, false, false> without the user line shape and chi, and its launcher.
#define MARFA_USER_PLUGINS 0
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f32, float, false, false, 4)
