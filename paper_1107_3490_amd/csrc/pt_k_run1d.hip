// pt_k_run1d.hip -- the persistent kernel for 1 wavefront(s) per replica, FP64 order.
#define PT_RUN_W 1
#define PT_RUN_MIXED false
#define PT_RUN_CAP run_cap_1d
#define PT_RUN_LAUNCH run_launch_1d
#include "pt_k_run.inc"
