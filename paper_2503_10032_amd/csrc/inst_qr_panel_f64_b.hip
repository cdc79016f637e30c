#include "inst_qr_panel.inc"
DDELM_INST_PANEL(double, 4, 512)
DDELM_INST_PANEL(double, 5, 512)
DDELM_INST_PANEL(double, 6, 512)
