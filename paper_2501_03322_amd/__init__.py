"""MI355X-native finite-source binary-lens magnification (contour integration).

The compute path is the HIP library built from csrc/ (libtwk.so); the Python
module `twk` is a thin ctypes binding of its C ABI (include/twk.h).
"""
