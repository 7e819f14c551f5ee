"""The real-space pair kernel evaluates erfc(x) as t P(t) exp(-x^2), with
t = 1/(1 + p x), from the FP32 coefficients in csrc/erfc_coeffs.h.  Here that
shipped table is checked on the host: it is what its generator writes, and it
matches scipy's erfc over the whole range the kernel uses (x = alpha r up to
3.5), both with the FP32 coefficients evaluated in FP64 and with every step
rounded to FP32 in order: the reciprocal for t, Horner's rule, the Gaussian and
the final products."""
import pathlib
import re
import subprocess
import sys

import numpy as np
from scipy.special import erfc, erfcx

CSRC = pathlib.Path(__file__).resolve().parents[1] / 'paper_2603_22274_amd' / 'csrc'
HEADER = CSRC / 'erfc_coeffs.h'


def _table():
    text = HEADER.read_text()
    p = float(re.search(r'FELIS_ERFC_P ([0-9.e+-]+)f', text).group(1))
    nc = int(re.search(r'FELIS_ERFC_NC (\d+)', text).group(1))
    c = [float(v) for v in re.findall(r'^\s+(-?[0-9.]+e[+-][0-9]+)f', text, re.M)]
    assert len(c) == nc
    return np.float32(p), np.array(c, dtype=np.float32)  # highest degree first


def test_header_is_what_the_generator_writes():
    out = subprocess.run([sys.executable, str(CSRC / 'gen_erfc_coeffs.py')],
                         capture_output=True, text=True, check=True, timeout=120).stdout
    assert out == HEADER.read_text()


def test_fp32_coefficients_in_fp64():
    p, c = _table()
    x = np.linspace(0.0, 3.5, 400_001)
    t = 1.0 / (1.0 + np.float64(p) * x)
    rel = t * np.polyval(c.astype(np.float64), t) / erfcx(x) - 1.0
    assert np.max(np.abs(rel)) <= 2e-7, np.max(np.abs(rel))
    # at x = 0 the fit reproduces erfc(0) = 1, so the coefficients sum to 1
    assert abs(float(c.astype(np.float64).sum()) - 1.0) <= 2e-7


def test_every_step_rounded_to_fp32():
    p, c = _table()
    f32 = np.float32
    x = np.linspace(0.0, 3.5, 400_001).astype(f32)
    t = (f32(1) / (f32(1) + p * x)).astype(f32)
    acc = np.zeros_like(t)
    for ci in c:
        acc = (acc * t + ci).astype(f32)
    g = np.exp(-(x * x)).astype(f32)
    e = (t * acc * g).astype(f32)
    rel = e.astype(np.float64) / erfc(x.astype(np.float64)) - 1.0
    # a few FP32 ulps: the rounding of t and of x^2 dominates near x = 3.5
    assert np.max(np.abs(rel)) <= 1.5e-6, np.max(np.abs(rel))
