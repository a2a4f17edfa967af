"""MI355X-native candidate-move evaluation engine for open-pit block
scheduling under geological uncertainty (C ABI in include/mps.h, HIP kernels
in csrc/, ctypes binding in binding.py)."""

__all__ = ["binding"]
