#include "inst_qr_panel.inc"
DDELM_INST_PANEL(float, 4, 512)
DDELM_INST_PANEL(float, 5, 512)
DDELM_INST_PANEL(float, 6, 512)
