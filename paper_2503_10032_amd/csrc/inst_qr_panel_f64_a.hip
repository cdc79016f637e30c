#include "inst_qr_panel.inc"
DDELM_INST_PANEL(double, 1, 256)
DDELM_INST_PANEL(double, 1, 512)
DDELM_INST_PANEL(double, 2, 512)
DDELM_INST_PANEL(double, 3, 512)
