#include "inst_qr_panel.inc"
DDELM_INST_PANEL(float, 1)
DDELM_INST_PANEL(float, 2)
DDELM_INST_PANEL(float, 3)
