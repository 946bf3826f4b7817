"""MI355X-native matrix-free SIPG multigrid (Cui & Kanschat, "Multilevel
Interior Penalty Methods on GPUs").

The compute path is the C-ABI library `libdgmg.so` built from `csrc/`
(hand-written HIP for gfx950); `dgmg` is its thin Python binding.  Importing
this package loads nothing; `from paper_2405_18982_amd import dgmg` loads the
library and fails loudly when it has not been built.
"""
