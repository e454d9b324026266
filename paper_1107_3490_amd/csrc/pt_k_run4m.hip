// pt_k_run4m.hip -- the persistent kernel for 4 wavefront(s) per replica, mixed precision.
#define PT_RUN_W 4
#define PT_RUN_MIXED true
#define PT_RUN_CAP run_cap_4m
#define PT_RUN_LAUNCH run_launch_4m
#include "pt_k_run.inc"
