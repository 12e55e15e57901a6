"""MI355X-native hot path of encrypted WiSARD training and inference
(Homomorphic WiSARDs, arXiv 2403.20190).

The arithmetic runs in HIP kernels for gfx950 behind the C ABI declared in
``include/hwisard.h``; :mod:`.hwisard` is the thin ctypes binding over it and
:mod:`.client` the client-side preprocessing and PD-act decode.
"""
