"""Exhaustive device check of the shortened arithmetic of Box-Muller.

The GPU computes the quotient of its logarithm and the two Box-Muller roots
with shorter sequences than the general correctly rounded division and
square root (no operand scaling or special-value fix-up).  The step
definition fixes those operations as IEEE binary32 division and square
root, so the shorter sequences must return the same bits on every argument
they can receive: every float m in [0.70, 1.42] for the quotient (the
folded mantissa of the logarithm's argument), zero and every float in
[2^-96, 64] for the root (its argument is -2 ln u <= 34).  The helper
library is built by __graft_entry__.build() from tests/helpers/math_check.hip.
"""
import ctypes
import os
import struct

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "helpers", "libmathcheck.so")


def bits(x: float) -> int:
    return struct.unpack("<I", struct.pack("<f", x))[0]


@pytest.fixture(scope="module")
def check():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    for f in (L.math_check_div, L.math_check_sqrt):
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_ulonglong),
                      ctypes.POINTER(ctypes.c_uint32)]
    return L


def run(fn, lo: int, hi: int):
    bad = ctypes.c_ulonglong()
    first = ctypes.c_uint32()
    rc = fn(lo, hi, ctypes.byref(bad), ctypes.byref(first))
    assert rc == 0, f"HIP error {rc}"
    return bad.value, first.value


def test_log_quotient_equals_ieee_division(check):
    # a margin beyond sqrt(1/2) and sqrt(2) on both sides
    lo, hi = bits(0.70), bits(1.42)
    print(f"division check over {hi - lo + 1} arguments", flush=True)
    bad, first = run(check.math_check_div, lo, hi)
    assert bad == 0, f"{bad} mismatches, first at m bits {first:#010x}"


def test_radius_root_equals_ieee_sqrt(check):
    lo, hi = bits(2.0 ** -96), bits(64.0)
    print(f"square-root check over {hi - lo + 2} arguments", flush=True)
    bad, first = run(check.math_check_sqrt, 0, 0)
    assert bad == 0, "sqrt(0) differs"
    bad, first = run(check.math_check_sqrt, lo, hi)
    assert bad == 0, f"{bad} mismatches, first at x bits {first:#010x}"
