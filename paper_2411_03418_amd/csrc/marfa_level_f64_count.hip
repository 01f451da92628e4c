// marfa_level_f64_count.hip -- k_level<double, true, false> and its launcher.
#include "marfa_level.h"

MARFA_LEVEL_LAUNCHER(launch_level_f64_count, double, true, false)
