"""The paper's cache-block and memory-traffic models, as printed (Sec. III-B, III-C).

TEST INFRASTRUCTURE ONLY (used by tests and the benchmark's reporting checks).

Notation (Sec. III-B): Dw diamond width along y, N_F wavefront frontlines,
N_xb bytes of the leading-dimension tile, R stencil radius, N_D number of
domain-sized streams (2 for 7c/25c, 9 for 7v, 15 for 25v).
"""
from __future__ import annotations


def wavefront_width_r1(Dw: float, NF: float) -> float:
    """W_w for a radius-1 stencil (Sec. III-B, before Eq. 2)."""
    return Dw + NF - 2


def cache_block_r1(Dw: float, NF: float, Nxb: float, ND: float) -> float:
    """Eq. (2): wavefront cache block size in bytes for R = 1."""
    Ww = wavefront_width_r1(Dw, NF)
    return Nxb * (ND * (Dw * Dw / 2 + Dw * (NF - 1)) + 2 * (Dw + Ww))


def wavefront_width(Dw: float, NF: float, R: float) -> float:
    """W_w for a general radius (Sec. III-B, before Eq. 3)."""
    return Dw - 2 * R + NF


def cache_block(Dw: float, NF: float, Nxb: float, R: float, ND: float) -> float:
    """Eq. (3): wavefront cache block size in bytes for a general radius."""
    Ww = wavefront_width(Dw, NF, R)
    return Nxb * (ND * Dw * (Dw / 2 - R + NF) + 2 * R * (Dw + Ww))


def code_balance_r1(Dw: float, ND: float) -> float:
    """Eq. (4): MWD code balance in bytes/LUP at double precision, R = 1."""
    return 16 * ((2 * Dw - 2) + (ND * Dw + 2)) / (Dw * Dw)


def code_balance(Dw: float, ND: float, R: float, elem_bytes: int = 8) -> float:
    """Eq. (5) in bytes/LUP; the printed constant 16 is two 8-byte words.

    ``elem_bytes`` = 4 restates the same traffic count for single precision.
    """
    return 2 * elem_bytes * R * ((2 * Dw - 2 * R) + (ND * Dw + 2 * R)) / (Dw * Dw)


ND = {"7c": 2, "7v": 9, "25c": 2, "25v": 15}
RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4}


def naive_code_balance(kind: str, elem_bytes: int) -> float:
    """Bytes per LUP of one full sweep when every stream is read or written once."""
    return elem_bytes * ND[kind]
