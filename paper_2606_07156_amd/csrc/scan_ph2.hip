// Scan kernels of phase 2 (see scan_kernels.h and scan_pick.inc).
#include "scan_kernels.h"
#define AMP_SCAN_PHASE 2
#include "scan_pick.inc"
