// FP32 instantiation of the stencil launchers (multigrid levels in FP32).
#define JFNK_T float
#include "ops_stencil.inc"
