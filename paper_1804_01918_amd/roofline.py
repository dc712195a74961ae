"""Algorithmic traffic and peak figures for the D2Q37 step on MI355X.

Bytes: every population of a site is read once and written once per step
(37 + 37 storage elements); a split propagate-then-collide pass moves each
population through HBM twice. Halo re-reads of neighbouring lines are not
algorithmic traffic.
"""
from __future__ import annotations

Q = 37
ELEM_BYTES = {"f64": 8, "f32": 4, "f16": 2}

# MI355X published peaks.
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
FP32_VECTOR_TFLOPS = 157.3
BF16_MFMA_TFLOPS = 2500.0


def bytes_per_site(dtype: str, fused: bool = True) -> int:
    b = 2 * Q * ELEM_BYTES[dtype]
    return b if fused else 2 * b


def roof_mlups(dtype: str, fused: bool = True, gbs: float = HBM_PEAK_GBS) -> float:
    return gbs * 1e9 / bytes_per_site(dtype, fused) / 1e6
