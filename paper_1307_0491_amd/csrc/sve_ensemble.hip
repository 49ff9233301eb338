// sve_ensemble.hip -- batched ensemble of independent runs (filled in below).
#include "sve_context.hpp"
