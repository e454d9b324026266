// pt_k_run2d.hip -- the persistent kernel for 2 wavefront(s) per replica, FP64 order.
#define PT_RUN_W 2
#define PT_RUN_MIXED false
#define PT_RUN_CAP run_cap_2d
#define PT_RUN_LAUNCH run_launch_2d
#include "pt_k_run.inc"
