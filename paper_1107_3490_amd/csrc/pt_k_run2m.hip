// pt_k_run2m.hip -- the persistent kernel for 2 wavefront(s) per replica, mixed precision.
#define PT_RUN_W 2
#define PT_RUN_MIXED true
#define PT_RUN_CAP run_cap_2m
#define PT_RUN_LAUNCH run_launch_2m
#include "pt_k_run.inc"
