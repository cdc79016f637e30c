#include "inst_cg_fused.inc"
DDELM_INST_CG(float, 1)
DDELM_INST_CG(float, 2)
DDELM_INST_CG(float, 4)
DDELM_INST_CG(float, 8)
DDELM_INST_CG(float, 16)
