"""The e4m11 storage format's conversions (the library's device functions,
compiled here as host code by a small harness) against an independent
numpy restatement of the format: every code decodes to the value its bit
fields define, and FP32 values -- every power-of-two boundary, the ties
halfway between neighbouring codes, the subnormal range, FP32 denormals, the
overflow threshold, the largest FP32 values, NaN and infinities, and random
values over the whole range --
encode to the nearest code with ties to even."""
import os
import subprocess

import numpy as np
import pytest

from parity_utils import E4M11_MAX, round_to_e4m11

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("e4m11") / "e4m11_harness")
    subprocess.run(["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "e4m11_harness.cpp"), "-o", exe], check=True)
    return exe


def _field_value(c):
    """Value of code c from its bit fields: sign, exponent E (4 bits),
    fraction M (11 bits); E = 0 subnormal M 2^-25, E = 15 infinity / NaN."""
    s = -1.0 if c >> 15 else 1.0
    E, M = (c >> 11) & 15, c & 0x7FF
    if E == 15:
        return s * np.inf if M == 0 else np.nan
    if E == 0:
        return s * M * 2.0 ** -25
    return s * 2.0 ** (E - 15) * (1 + M / 2048)


def test_every_code_decodes_to_its_value(harness, tmp_path):
    out = tmp_path / "dec.f32"
    subprocess.run([harness, "decode", str(out)], check=True)
    with np.errstate(invalid="ignore"):
        got = np.fromfile(out, dtype=np.float32).astype(np.float64)
    want = np.array([_field_value(c) for c in range(65536)])
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], want[~nan])
    assert np.array_equal(np.signbit(got[~nan]), np.signbit(want[~nan]))  # -0 stays -0
    assert got[0x77FF] == E4M11_MAX


def _codes_of_values(v):
    """Code of each representable value v (inverse of the field decoding)."""
    table = {}
    for c in range(65536):
        x = _field_value(c)
        if not np.isnan(x):
            table[(np.signbit(x), abs(x))] = c
    return np.array([table[(np.signbit(x), abs(x))] for x in v])


def test_encode_rounds_to_nearest_even(harness, tmp_path):
    rng = np.random.default_rng(5)
    reps = np.array([_field_value(c) for c in range(0x7800)])  # all finite non-negative values
    mids = (reps[:-1] + reps[1:]) / 2  # exact ties (representable in FP32)
    xs = [reps, mids, np.nextafter(mids.astype(np.float32), np.float32(0)).astype(np.float64),
          np.nextafter(mids.astype(np.float32), np.float32(1)).astype(np.float64),
          rng.uniform(0, 1, 200000), 10.0 ** rng.uniform(-12, 0, 200000),
          [2.0 ** -26, 2.0 ** -26 * (1 + 2 ** -23), 2.0 ** -27, 1e-30, 0.0,
           E4M11_MAX, (E4M11_MAX + 1.0) / 2, np.nextafter(np.float32((E4M11_MAX + 1.0) / 2), 0),
           1.0, 3.5, 1e30,
           # FP32 denormals, and magnitudes around 2^116, where the rounding
           # constant of the encoder leaves the FP32 range
           1e-40, 2.0 ** -149, 2.0 ** -126, 2.0 ** 115, 2.0 ** 116, 2.0 ** 120,
           float(np.finfo(np.float32).max)]]
    x = np.concatenate([np.asarray(a, dtype=np.float64) for a in xs]).astype(np.float32)
    x = np.concatenate([x, -x])
    assert np.all(np.isfinite(x))
    src, dst = tmp_path / "in.f32", tmp_path / "out.u16"
    x.tofile(src)
    subprocess.run([harness, "encode", str(src), str(dst)], check=True)
    got = np.fromfile(dst, dtype=np.uint16).astype(np.int64)
    want_val = round_to_e4m11(x.astype(np.float64))
    finite = np.isfinite(want_val)
    assert np.array_equal(got[finite], _codes_of_values(want_val[finite]))
    assert np.all(got[~finite] & 0x7FFF == 0x7800)  # past the largest finite: infinity
    assert np.array_equal(got[~finite] >> 15, np.signbit(x[~finite]).astype(np.int64))
    # ties went to the even code
    tie_codes = got[len(reps):len(reps) + len(mids)]
    assert np.all(tie_codes % 2 == 0)


def test_non_finite_inputs(harness, tmp_path):
    x = np.array([np.inf, -np.inf, np.nan], dtype=np.float32)
    src, dst = tmp_path / "in.f32", tmp_path / "out.u16"
    x.tofile(src)
    subprocess.run([harness, "encode", str(src), str(dst)], check=True)
    got = np.fromfile(dst, dtype=np.uint16)
    assert got[0] == 0x7800 and got[1] == 0xF800
    assert (got[2] >> 11) & 15 == 15 and got[2] & 0x7FF != 0
