// pt_k_run1m.hip -- the persistent kernel for 1 wavefront(s) per replica, mixed precision.
#define PT_RUN_W 1
#define PT_RUN_MIXED true
#define PT_RUN_CAP run_cap_1m
#define PT_RUN_LAUNCH run_launch_1m
#include "pt_k_run.inc"
