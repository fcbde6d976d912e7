"""The generated FFT codelets, evaluated on the CPU (no GPU needed).

Every codelet of gen_fft.py is straight-line code over a handful of complex
helpers; here each line is evaluated with Python complex numbers and the result
compared with numpy's FFT: run() is the unnormalised DFT with sign s
(v[k] <- sum_j v[j] exp(s 2 pi i jk / n)) and tw2() multiplies v[j] by
exp(s 2 pi i j / (2n)), for every length the kernels instantiate.
"""
import importlib.util
import os
import re

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GEN = os.path.join(HERE, "..", "paper_2506_20350_amd", "csrc", "gen_fft.py")

_spec = importlib.util.spec_from_file_location("gen_fft", GEN)
gen_fft = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(gen_fft)

OPS = {
    "cadd": lambda a, b: a + b,
    "csub": lambda a, b: a - b,
    "cneg": lambda a: -a,
    "cmuli": lambda a: 1j * a,
    "cmulni": lambda a: -1j * a,
    "cscale": lambda a, c: a * c,
    "cfmar": lambda a, c, b: a * c + b,
    "cmulc": lambda a, c, s: a * complex(c, s),
    "R": float,
}


def _bodies(n, s):
    text = gen_fft.codelet(n, s)
    run = text[text.index("void run(C* v) {"):text.index("static __device__ __forceinline__ void tw2")]
    tw2 = text[text.index("void tw2(C* v) {"):]
    return run, tw2


def _evaluate(body, v):
    env = dict(OPS)
    env["v"] = list(v)
    for line in body.splitlines():
        line = line.strip()
        m = re.match(r"const C (t\d+) = (.*);$", line)
        if m:
            env[m.group(1)] = eval(m.group(2), {}, env)
            continue
        m = re.match(r"v\[(\d+)\] = (.*);$", line)
        if m:
            env["v"][int(m.group(1))] = eval(m.group(2).replace("czero<C>()", "0j"), {}, env)
    return np.array(env["v"])


@pytest.mark.parametrize("n", list(range(1, 33)))
@pytest.mark.parametrize("s", [-1, 1])
def test_codelet_is_the_dft_and_tw2_the_half_twiddle(n, s):
    rng = np.random.default_rng(n * 7 + (s > 0))
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    run, tw2 = _bodies(n, s)
    ref = np.fft.fft(x) if s < 0 else np.fft.ifft(x) * n
    got = _evaluate(run, x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    j = np.arange(n)
    got2 = _evaluate(tw2, x)
    np.testing.assert_allclose(got2, x * np.exp(s * 2j * np.pi * j / (2 * n)), rtol=0, atol=1e-13)
