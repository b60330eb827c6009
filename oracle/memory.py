"""Field-memory formulas of Section 3.3 (bytes), as the paper states them.

* Hockney-Eastwood: five float64 fields on (2N)^3, three 4-byte integer
  fields on (2N)^3, one float64 field on N^3 (rho reused for phi).
* Vico-Greengard (original): the same without the integer fields, plus two
  float64 fields on (4N)^3.
* Modified Vico-Greengard (DCT): as Vico-Greengard but one float64 field on
  (2N+1)^3 instead of the two (4N)^3 fields.
"""
from __future__ import annotations

__all__ = ["hockney_bytes", "vico_bytes", "vico_dct_bytes"]


def hockney_bytes(n: int) -> int:
    return 5 * (2 * n) ** 3 * 8 + 3 * (2 * n) ** 3 * 4 + n ** 3 * 8


def vico_bytes(n: int) -> int:
    return 5 * (2 * n) ** 3 * 8 + n ** 3 * 8 + 2 * (4 * n) ** 3 * 8


def vico_dct_bytes(n: int) -> int:
    return 5 * (2 * n) ** 3 * 8 + n ** 3 * 8 + (2 * n + 1) ** 3 * 8
