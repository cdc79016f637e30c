#include "inst_qr_panel.inc"
DDELM_INST_PANEL(float, 1, 256)
DDELM_INST_PANEL(float, 1, 512)
DDELM_INST_PANEL(float, 2, 512)
DDELM_INST_PANEL(float, 3, 512)
