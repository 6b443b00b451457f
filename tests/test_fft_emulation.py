"""The library's in-LDS FFT stages (csrc/fft_core.h) run on the CPU: the
header is built by the host compiler against a stand-in for the HIP runtime
(tests/host/hipshim) with one std::thread per GPU thread and a std::barrier
for the block barrier (tests/host/fft_emulate.cpp), under AddressSanitizer.
Every supported length is checked against numpy's FFT in both directions,
in the two layouts the kernels use (elements contiguous with lines at an odd
pitch; lines contiguous with elements at a pitch), on part of the lines; the
row-listed transform (lds_fft_rows, butterflies dealt over the listed lines
only) on scattered line lists; and the fused inverse / multiply / forward
pair (lds_fft_pair) against ifft, multiply, fft.  Lines the call must not
touch and the padding of every line hold NaN-free sentinels that must come
back unchanged."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DRIVER = os.path.join(HERE, "host", "fft_emulate.cpp")
LENGTHS = [8, 12, 16, 18, 20, 24, 30, 32, 36, 40, 48, 60, 64, 72, 80, 90, 96, 100, 108, 120, 128]
PAIR_LENGTHS = [n for n in LENGTHS if n not in (90, 100, 120)]   # one or two stages
FLOAT_LENGTHS = [48, 60, 108]
MAXL_FFT, MAXL_PAIR = 12, 10
SENTINEL = 12345.0 - 678.0j


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("fftemu") / "fft_emulate")
    cmd = [gxx, "-std=c++20", "-O0", "-fno-omit-frame-pointer", "-pthread",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + os.path.join(HERE, "host", "hipshim"),
           "-I" + os.path.join(ROOT, "paper_2505_02319_amd", "csrc"), DRIVER, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]

    def run(lines):
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
        p = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True,
                           text=True, env=env, timeout=600)
        assert p.returncode == 0, p.stderr[-4000:]
        assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr[-4000:]
        out = []
        for ln in p.stdout.splitlines():
            v = np.array([float(t) for t in ln.split()])
            out.append(v[0::2] + 1j * v[1::2])
        assert len(out) == len(lines)
        return out
    return run


def r(x):
    return repr(float(x))


def cbuf(b):
    return f"{len(b)} " + " ".join(f"{r(z.real)} {r(z.imag)}" for z in b)


def layout(n, maxl, transposed):
    """(lstride, estride, buffer length) of maxl lines of n elements."""
    if transposed:
        return 1, maxl + 1, n * (maxl + 1)
    return n + 1, 1, maxl * (n + 1)


def lines_of(buf, n, lines, ls, es):
    return np.array([[buf[l * ls + e * es] for e in range(n)] for l in lines])


def prec_tol(prec, n):
    return (1e-13 if prec == 0 else 2e-6) * max(1.0, np.log2(n))


def test_line_transforms_all_lengths(emu):
    rng = np.random.default_rng(21)
    cases, meta = [], []
    for n in LENGTHS:
        for inv in (0, 1):
            for transposed in (False, True):
                for prec in ((0, 1) if n in FLOAT_LENGTHS else (0,)):
                    nl = int(rng.integers(1, MAXL_FFT + 1)) if transposed else MAXL_FFT - 1
                    ls, es, blen = layout(n, MAXL_FFT, transposed)
                    buf = np.full(blen, SENTINEL)
                    x = rng.standard_normal((nl, n)) + 1j * rng.standard_normal((nl, n))
                    for l in range(nl):
                        for e in range(n):
                            buf[l * ls + e * es] = x[l, e]
                    cases.append(f"fft {prec} {n} {inv} {nl} {ls} {es} {cbuf(buf)}")
                    meta.append((n, inv, nl, ls, es, buf, x, prec))
    for got, (n, inv, nl, ls, es, buf, x, prec) in zip(emu(cases), meta):
        want = np.fft.ifft(x, axis=1) * n if inv else np.fft.fft(x, axis=1)
        y = lines_of(got, n, range(nl), ls, es)
        err = np.max(np.abs(y - want)) / np.max(np.abs(want))
        assert err < prec_tol(prec, n), (n, inv, ls, es, prec, err)
        touched = np.zeros(len(buf), bool)
        for l in range(nl):
            for e in range(n):
                touched[l * ls + e * es] = True
        assert np.array_equal(got[~touched], buf[~touched]), (n, inv, "untouched entries changed")


def test_row_listed_transforms(emu):
    """lds_fft_rows: the listed lines (scattered, any count up to MAXL) are
    transformed, the others come back unchanged."""
    rng = np.random.default_rng(22)
    cases, meta = [], []
    for n in LENGTHS:
        for inv in (0, 1):
            for prec in ((0, 1) if n in FLOAT_LENGTHS else (0,)):
                for nl in (1, 5, MAXL_FFT - 3, MAXL_FFT):
                    rows = np.sort(rng.choice(MAXL_FFT, size=nl, replace=False))
                    ls, es, blen = layout(n, MAXL_FFT, False)
                    buf = (rng.standard_normal(blen) + 1j * rng.standard_normal(blen))
                    if prec == 1:                     # inputs exact in FP32
                        buf = buf.astype(np.complex64).astype(np.complex128)
                    buf[n::ls] = SENTINEL             # padding element of every line
                    lm = " ".join(str(int(v)) for v in rows)
                    cases.append(f"rows {prec} {n} {inv} {nl} {ls} {es} {lm} {cbuf(buf)}")
                    meta.append((n, inv, rows, ls, es, buf, prec))
    for got, (n, inv, rows, ls, es, buf, prec) in zip(emu(cases), meta):
        x = lines_of(buf, n, rows, ls, es)
        want = np.fft.ifft(x, axis=1) * n if inv else np.fft.fft(x, axis=1)
        y = lines_of(got, n, rows, ls, es)
        err = np.max(np.abs(y - want)) / np.max(np.abs(want))
        assert err < prec_tol(prec, n), (n, inv, list(rows), prec, err)
        others = [l for l in range(MAXL_FFT) if l not in set(rows.tolist())]
        assert np.array_equal(lines_of(got, n, others, ls, es), lines_of(buf, n, others, ls, es))
        assert np.array_equal(got[n::ls], buf[n::ls])


def test_transform_pair_with_multiply(emu):
    """lds_fft_pair: per line, fft(s * ifft(x) * N), the last inverse stage,
    the multiply and the first forward stage fused in registers."""
    rng = np.random.default_rng(23)
    cases, meta = [], []
    for n in PAIR_LENGTHS:
        for transposed in (True, False):
            for prec in ((0, 1) if n in FLOAT_LENGTHS else (0,)):
                ls, es, blen = layout(n, MAXL_PAIR, transposed)
                buf = np.full(blen, SENTINEL)
                x = rng.standard_normal((MAXL_PAIR, n)) + 1j * rng.standard_normal((MAXL_PAIR, n))
                for l in range(MAXL_PAIR):
                    for e in range(n):
                        buf[l * ls + e * es] = x[l, e]
                s = rng.uniform(-2, 2, (MAXL_PAIR, n))
                cases.append(f"pair {prec} {n} {ls} {es} {' '.join(r(v) for v in s.ravel())} "
                             f"{cbuf(buf)}")
                meta.append((n, ls, es, buf, x, s, prec))
    for got, (n, ls, es, buf, x, s, prec) in zip(emu(cases), meta):
        want = np.fft.fft(s * (np.fft.ifft(x, axis=1) * n), axis=1)
        y = lines_of(got, n, range(MAXL_PAIR), ls, es)
        err = np.max(np.abs(y - want)) / np.max(np.abs(want))
        assert err < prec_tol(prec, n), (n, ls, es, prec, err)
        touched = np.zeros(len(buf), bool)
        for l in range(MAXL_PAIR):
            for e in range(n):
                touched[l * ls + e * es] = True
        assert np.array_equal(got[~touched], buf[~touched])
