// marfa_level_f64.hip -- k_level<double, false, false> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(launch_level_f64, double, false, false)
