// pt_k_run4d.hip -- the persistent kernel for 4 wavefront(s) per replica, FP64 order.
#define PT_RUN_W 4
#define PT_RUN_MIXED false
#define PT_RUN_CAP run_cap_4d
#define PT_RUN_LAUNCH run_launch_4d
#include "pt_k_run.inc"
