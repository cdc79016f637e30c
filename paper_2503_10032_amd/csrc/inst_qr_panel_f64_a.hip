#include "inst_qr_panel.inc"
DDELM_INST_PANEL(double, 1)
DDELM_INST_PANEL(double, 2)
DDELM_INST_PANEL(double, 3)
