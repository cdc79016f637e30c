#include "inst_qr_panel.inc"
DDELM_INST_PANEL(double, 4)
DDELM_INST_PANEL(double, 5)
DDELM_INST_PANEL(double, 6)
