// marfa_level_f64.hip -- the level kernel <double, false, false> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f64, double, false, false, 1)
