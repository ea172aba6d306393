"""MI355X-native time stepper of the Fullwave 2 nonlinear acoustic system
(Sode & Pinton, arXiv 2106.11476): a C-ABI HIP library (libfw2.so, include/fw2.h)
and its thin Python binding (paper_2106_11476_amd.fw2)."""
