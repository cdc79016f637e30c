#include "inst_cg_fused.inc"
DDELM_INST_CG(double, 1)
DDELM_INST_CG(double, 2)
DDELM_INST_CG(double, 4)
DDELM_INST_CG(double, 8)
DDELM_INST_CG(double, 16)
