#include "inst_qr_panel.inc"
DDELM_INST_PANEL(float, 4)
DDELM_INST_PANEL(float, 5)
DDELM_INST_PANEL(float, 6)
