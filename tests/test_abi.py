"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/nshe.h declares, rejects bad parameters before it
touches a device, and the package's default parameters equal the oracle's
independently derived ones."""
import ctypes
import os
import re

import pytest

from paper_2602_24271_amd import _lib, params
from oracle import nt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("nshe.h", "nshe_probe.h")]


def _declared():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nshe_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_expected_calls():
    names = _declared()
    for must in ("nshe_ctx_create", "nshe_set_relin_key", "nshe_sub", "nshe_square_relin",
                 "nshe_mul_relin", "nshe_eq_mask", "nshe_eq_mask_batched", "nshe_margin_events",
                 "nshe_last_error", "nshe_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding describes every one of them
    assert set(_declared()) == set(_lib.SIGNATURES)


def _create(log2_n=10, t=65537, q=None, P=None):
    lib = _lib.load()
    if q is None:
        q, P = params.modulus_chain()
    qa = (ctypes.c_uint64 * len(q))(*q)
    pr = _lib.NsheParams(log2_n, t, len(q), ctypes.cast(qa, ctypes.POINTER(ctypes.c_uint64)), P)
    h = ctypes.c_void_p()
    rc = lib.nshe_ctx_create(ctypes.byref(pr), 0, ctypes.byref(h))
    return rc, lib.nshe_last_error().decode(), h


@pytest.mark.parametrize("kw,msg", [
    (dict(log2_n=2), "log2_n"),
    (dict(log2_n=16), "log2_n"),
    (dict(t=65536), "t must be odd"),
    (dict(t=1), "t must be odd"),
    (dict(q=[97, 193], P=257), "[2^48, 2^49)"),
])
def test_create_rejects_bad_parameters_before_device_use(kw, msg):
    rc, err, h = _create(**kw)
    assert rc == -1 and msg in err and not h.value


def test_create_rejects_unsupported_prime_counts():
    q, P = params.modulus_chain()
    for L in (1, 5, 18):
        rc, err, h = _create(q=q[:L] if L <= len(q) else q + q[:1], P=P)
        assert rc == -1 and not h.value
        assert "L must be one of" in err


def test_create_rejects_composite_and_duplicate_primes():
    q, P = params.modulus_chain()
    rc, err, _ = _create(q=[q[0] + 65536 * 3] + q[1:], P=P)  # 1 mod 2^16, composite or not prime
    if nt.is_prime(q[0] + 65536 * 3):
        pytest.skip("perturbed value happens to be prime")
    assert rc == -1 and "not prime" in err
    rc, err, _ = _create(q=[q[0], q[0]] + q[2:], P=P)
    assert rc == -1 and "distinct" in err


def test_null_arguments_are_rejected():
    lib = _lib.load()
    assert lib.nshe_ctx_create(None, 0, None) == -1
    assert lib.nshe_sub(None, None, None, None, 1, None) == -1
    assert lib.nshe_workspace_bytes(None, 4) == 0
    assert lib.nshe_eq_mask(None, None, None, None, 1, 0, None, 0, None) == -1


def test_default_parameters_match_the_oracle():
    q, P = params.modulus_chain()
    oq, oP = nt.default_modulus_chain()
    assert (q, P) == (oq, oP)


def test_noalloc_scratch_is_a_global_device_symbol(tmp_path):
    """The no-allocation entry point's scratch array must be a global symbol
    of the device code object: the runtime finds registered device variables
    by name among global symbols when it loads the code (a local one is not
    found).  Checked on the built library with the ROCm LLVM tools."""
    import shutil
    import subprocess
    objdump = "/opt/rocm/llvm/bin/llvm-objdump"
    readelf = "/opt/rocm/llvm/bin/llvm-readelf"
    if not (os.path.exists(objdump) and os.path.exists(readelf)):
        pytest.skip("ROCm LLVM tools not installed")
    lib = tmp_path / "libnshe.so"
    shutil.copy(_lib.LIB_PATH, lib)
    subprocess.run([objdump, "--offloading", str(lib)], cwd=tmp_path, capture_output=True,
                   check=True)
    found = []
    for f in sorted(tmp_path.glob("libnshe.so.*gfx950")):
        out = subprocess.run([readelf, "-s", "--wide", str(f)], capture_output=True, text=True,
                             check=True).stdout
        found += [line.split() for line in out.splitlines() if line.endswith("_ZL7scratch")]
    assert found, "no scratch symbol in the device code"
    # (the static and the dynamic symbol tables may both list it)
    assert {(int(f[2]), f[3], f[4]) for f in found} == {(160 << 20, "OBJECT", "GLOBAL")}, found


def _create2(log2_n=10, L=16, P1=None):
    lib = _lib.load()
    q, (P0, P1d) = params.modulus_chain(n_special=2)
    q = q[:L]
    qa = (ctypes.c_uint64 * len(q))(*q)
    pr = _lib.NsheParams(log2_n, 65537, len(q), ctypes.cast(qa, ctypes.POINTER(ctypes.c_uint64)),
                         P0, 2, P1d if P1 is None else P1)
    h = ctypes.c_void_p()
    rc = lib.nshe_ctx_create(ctypes.byref(pr), 0, ctypes.byref(h))
    return rc, lib.nshe_last_error().decode(), h


def test_two_special_primes_parameter_rules():
    """alpha = 2 needs an even supported L and a valid, distinct second
    special prime; rejected on the host before any device use."""
    rc, err, h = _create2(L=12)
    assert rc == -1 and "alpha = 2" in err and not h.value
    q, P = params.modulus_chain()
    rc, err, h = _create2(P1=q[3])
    assert rc == -1 and "distinct" in err and not h.value
    rc, err, h = _create2(P1=97)
    assert rc == -1 and "[2^48, 2^49)" in err and not h.value


def test_two_special_primes_match_the_oracle():
    q, sp = params.modulus_chain(n_special=2)
    oq, osp = nt.default_modulus_chain(n_special=2)
    assert (q, sp) == (oq, osp) and len(q) == 16


def test_three_special_primes_parameter_rules():
    lib = _lib.load()
    q, sp = params.modulus_chain(n_special=3)
    assert len(q) == 15 and len(sp) == 3
    for L, ok in ((15, True), (16, False)):
        qq = (q + list(params.modulus_chain()[0]))[:L] if L > 15 else q[:L]
        qa = (ctypes.c_uint64 * len(qq))(*qq)
        pr = _lib.NsheParams(15, 65537, len(qq), ctypes.cast(qa, ctypes.POINTER(ctypes.c_uint64)),
                             sp[0], 3, sp[1], sp[2])
        b = _lib.NsheBudget()
        rc = lib.nshe_budget_of(ctypes.byref(pr), ctypes.byref(b))
        if ok:
            assert rc == 0 and b.depth_budget == 21
        else:
            assert rc == -1 and "alpha = 3" in lib.nshe_last_error().decode()


# C struct name -> (ctypes class, field names): the binding's structs must have the header's
# size and field offsets (checked by compiling a C program against the header with gcc)
_STRUCTS = {
    "nshe_params": ("NsheParams", ["log2_n", "t", "L", "q_host", "P", "alpha", "P1", "P2"]),
    "nshe_info": ("NsheInfo", ["n", "L", "L_ext", "squarings", "ext_primes", "ct_words",
                               "relin_key_words", "depth_budget", "lt_depth", "fresh_bits",
                               "level_bits", "alpha", "dnum"]),
    "nshe_budget": ("NsheBudget", ["depth_budget", "lt_depth", "fresh_bits", "level_bits"]),
    "nshe_item": ("NsheItem", ["x_dev", "y_dev", "out_dev", "n_ct", "y_broadcast"]),
    "nshe_tuning": ("NsheTuning", ["ks_chunk", "split_forward", "ew_block", "wave_ct",
                                   "ks_fused", "streams"]),
    "nshe_kernel_stat": ("NsheKernelStat", ["name", "launches", "total_ms", "work"]),
    "nshe_modmul_probe": ("NsheModmulProbe", ["ms", "products_per_s", "fp64_ops_per_s"]),
    "nshe_conv_probe": ("NsheConvProbe", ["coefficients", "ms_fma", "ms_mfma", "mismatches"]),
    "nshe_overlap_probe": ("NsheOverlapProbe", ["ms_valu", "ms_mfma", "ms_both", "fma_per_s_valu",
                                                "fma_per_s_mfma"]),
}


def test_binding_structs_match_the_header(tmp_path):
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "nshe.h"',
             '#include "nshe_probe.h"', 'int main(void) {']
    for cname, (_, fields) in _STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, (pyname, fields) in _STRUCTS.items():
        cls = getattr(_lib, pyname)
        assert ctypes.sizeof(cls) == got[(cname, "size")], cname
        assert [f[0] for f in cls._fields_] == fields, cname
        for f in fields:
            assert getattr(cls, f).offset == got[(cname, f)], (cname, f)
