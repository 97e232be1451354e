// Scan kernels of phase 3 (see scan_kernels.h and scan_pick.inc).
#include "scan_kernels.h"
#define AMP_SCAN_PHASE 3
#include "scan_pick.inc"
