"""CPU checks of the C ABI: the built library loads and exports every function the header declares.

No compute call is made (there is no GPU on this host).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastlsq.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(flsq_[a-z_A-Z0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("flsq_solve_linear", "flsq_factorize", "flsq_factor_solve", "flsq_evaluate", "flsq_solve_newton",
                 "flsq_gram", "flsq_inverse_loss_grad"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2602_10541_amd import fastlsq
    if not os.path.exists(fastlsq.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(fastlsq.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) == set(fastlsq.EXPORTS)
    assert b"gfx950" in fastlsq.load().flsq_build_info()


def test_binding_structs_match_header_layout(tmp_path):
    """ctypes mirrors of the ABI structs have the sizes and field offsets that a C compiler
    gives the header's declarations."""
    import shutil
    import subprocess
    from paper_2602_10541_amd import fastlsq as fl
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = ["flsq_term", "flsq_op", "flsq_basis", "flsq_rows", "flsq_solve_opts", "flsq_solve_info",
               "flsq_newton_opts", "flsq_nonlin", "flsq_channel", "flsq_vrows", "flsq_nonlin_grad"]
    structs = [n for n in structs if hasattr(fl, n)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fastlsq.h"', "int main(void) {"]
    for n in structs:
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for f, _ in getattr(fl, n)._fields_:
            lines.append(f'  printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            *key, v = ln.split()
            got[tuple(key)] = int(v)
    for n in structs:
        cls = getattr(fl, n)
        assert ctypes.sizeof(cls) == got[(n, "size")], n
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == got[(n, f)], (n, f)


def test_no_gpu_means_loud_failure():
    """Without a GPU the binding raises; it never falls back to the CPU."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2602_10541_amd import fastlsq
    if not os.path.exists(fastlsq.LIB_PATH):
        pytest.skip("library not built")
    with pytest.raises(RuntimeError):
        fastlsq.Context(0)


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with a message before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_int8_residue_byte_identity():
    """The residue bytes of k_i8_residues (csrc/k_gram_i8.hip): for an integer a with
    |a| <= 2^46 and each modulus p of the int8 CRT set, q = low word of fma(a, 1/p, 1.5 * 2^52)
    and a_lo = low word of a + 1.5 * 2^52 give (a_lo + (256 - p) (q mod 2^24)) mod 256, which
    must be the two's-complement byte of the balanced residue a - p rint(a / p).  The fma is
    emulated exactly (one rounding of the exact rational), on random a and on the edge cases
    (0, +-2^46, values next to multiples of p and to the half-way points)."""
    import random
    import struct
    from fractions import Fraction
    from pathlib import Path
    src = (Path(__file__).resolve().parents[1] / "paper_2602_10541_amd" / "csrc" / "fastlsq.cpp").read_text()
    moduli = [int(v) for v in re.search(r"const int list\[13\] = \{([0-9, ]+)\}", src).group(1).split(",")]
    assert len(moduli) == 13
    bias = 6755399441055744.0

    def low_word(x):
        return struct.unpack("<Q", struct.pack("<d", x))[0] & 0xffffffff

    rng = random.Random(7)
    lim = 1 << 46
    values = [0, lim, -lim, lim - 1, -lim + 1] + [rng.randint(-lim, lim) for _ in range(600)]
    for p in moduli:
        for k in (1, 3, 12345, (lim // p) - 1):
            for s in (-1, 1):
                base = s * k * p
                values += [base + (p - 1) // 2, base - (p - 1) // 2, base + (p + 1) // 2, base - (p + 1) // 2]
    values = [v for v in values if abs(v) <= lim]
    for p in moduli:
        ip = 1.0 / p
        for a in values:
            q = low_word(float(Fraction(a) * Fraction(ip) + Fraction(bias)))
            a_lo = low_word(float(Fraction(a) + Fraction(bias)))
            got = (a_lo + (256 - p) * (q & 0xffffff)) & 0xff
            r = a - p * round(Fraction(a, p))
            assert 2 * abs(r) < p
            assert got == r & 0xff, (p, a, got, r)
