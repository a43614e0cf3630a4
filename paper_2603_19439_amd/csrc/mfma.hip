// BF16 MFMA kernels (filled in below)
#include "grest_internal.h"
