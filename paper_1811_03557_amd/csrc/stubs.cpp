// Entry points whose implementation is not built yet: they validate nothing and report it.
#include "common.h"

using namespace dpm;

