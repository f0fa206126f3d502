"""Batched ranged random integers on MI355X (gfx950).

Brackett-Rozinsky and Lemire, "Batched Ranged Random Integer Generation":
several unbiased bounded integers from one 64-bit word by a chain of
full-width multiplies and one rejection test on the leftover (Theorem 1),
feeding dice streams, Fisher-Yates shuffles and sampling without
replacement. The computation lives in libbrr.so (HIP kernels behind the C ABI
of include/brr.h); ``brr`` is its thin binding.
"""
__all__ = ["brr", "workloads"]
