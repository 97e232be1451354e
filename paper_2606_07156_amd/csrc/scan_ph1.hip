// Scan kernels of phase 1 (see scan_kernels.h and scan_pick.inc).
#include "scan_kernels.h"
#define AMP_SCAN_PHASE 1
#include "scan_pick.inc"
