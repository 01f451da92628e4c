// marfa_level_f64_count.hip -- the level kernel <double, true, false> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(f64_count, double, true, false, 1)
