"""Host logic of bench.py (no GPU): the refusal of more than one GPU, the
roofline op models checked against counts derived here from the workload's
shape, and the profile summary's counter calibration."""
import csv
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N = 1 << 15
CT = 32           # ciphertexts of the 2^20-row column
L, LB, A = 15, 16, 3
DNUM = L // A
K = L + A


def _ctx(split=1):
    return SimpleNamespace(n=N, L=L, L_ext=LB, alpha=A, dnum=DNUM,
                           tuning=lambda: {"split_forward": split, "ks_chunk": 32})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_scale_roofline_counts_two_conversions_per_tensor_coefficient():
    # a launch covers the three tensor components of every ciphertext
    coeffs = 3 * CT * N
    ms = 0.378
    prof = {"scale": {"launches": 16, "ms": 16 * ms, "work": 16 * coeffs}}
    r = bench.roofline_scale(prof, _ctx())
    # two conversions (L -> L + 1 and L + 1 -> L primes), L (L + 1) terms each,
    # four FP64 FMAs per term on 24-bit halves
    assert r["ops_per_launch"] == coeffs * 2 * L * LB * 4 == 6039797760
    assert r["frac"] == pytest.approx(6039797760 / (ms * 1e-3) / (256 * 64 * 2.4e9))
    assert r["peak"] == pytest.approx(39.3216)


def test_digit_roofline_counts_parity_stages_and_digit_values():
    # 32 ciphertexts x 5 digits x 18 primes = 2880 limbs, each by parity two
    # 2^14-point transforms of 14 stages (N/2 butterflies per stage)
    limbs = CT * DNUM * K
    bfly = limbs * (N // 2) * 14
    ms = 0.357
    prof = {"ntt_digit": {"launches": 16, "ms": 16 * ms, "work": 16 * bfly},
            "scale": {"launches": 16, "ms": 16 * 0.3, "work": 16}}
    r, kind = bench.roofline(prof, _ctx())
    assert kind == "ntt_digit" and r["stages_per_limb"] == 14
    assert r["butterflies_per_launch"] == bfly == 660602880
    # forming a three-prime digit's value: two exact products and additions
    # (7 FP64 operations each) per coefficient of every limb
    assert r["modup_ops_per_launch"] == limbs * N * 7 * 2 == 1321205760
    assert r["frac"] == pytest.approx((bfly * 8 + limbs * N * 14) / (ms * 1e-3) / 39.3216e12)
    # the full-limb transforms: 15 stages
    r1, _ = bench.roofline(prof, _ctx(split=0))
    assert r1["stages_per_limb"] == 15


def test_dominant_kind_picks_the_kernel_with_the_most_time():
    prof = {"scale": {"launches": 16, "ms": 6.0, "work": 16 * 3 * CT * N},
            "ntt_digit": {"launches": 16, "ms": 5.6, "work": 16 * 660602880},
            "ks_mac": {"launches": 16, "ms": 3.2, "work": 1.0}}
    dom, ntt = bench.roofline_dominant(prof, _ctx())
    assert dom["kernel"] == "scale" and ntt["kernel"] == "ntt_digit"
    prof["ntt_digit"]["ms"] = 7.0
    dom, ntt = bench.roofline_dominant(prof, _ctx())
    assert dom is ntt and dom["kernel"] == "ntt_digit"


def test_key_switch_product_bytes():
    ms = 0.2
    prof = {"ks_mac": {"launches": 16, "ms": 16 * ms, "work": 1.0}}
    r = bench.roofline_ks(_ctx(), prof, CT, 32)
    limb = 8 * N
    # digits read once; the key (dnum x 2 components) once per 16 ciphertexts
    # (the parity product's chunk); two sums written per ciphertext
    want = limb * K * (CT * DNUM + 2 * DNUM * 2 + CT * 2)
    assert r["bytes_per_launch"] == want == 1151336448
    assert r["frac"] == pytest.approx(want / (ms * 1e-3) / 8e12)
    # a chunk narrows to the ciphertexts present
    r8 = bench.roofline_ks(_ctx(), prof, 8, 32)
    assert r8["bytes_per_launch"] == limb * K * (8 * DNUM + 1 * DNUM * 2 + 8 * 2)


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_profile_summary_scales_counters_by_the_copy(tmp_path):
    """A 256 MiB device copy that FETCH_SIZE reads as half its size and
    WRITE_SIZE as its size: the factors are 2 and 1, and a kernel's bytes per
    launch are its mean counter value (KiB) times 1024 times the factor."""
    prof = tmp_path / "prof"
    scale = "void nshe::k_scale<15, true, 3>(int, unsigned long, double*, nshe::Tables)"
    digit = "void nshe::k_ntt_fwd_par<6, true>(nshe::NttJob, nshe::Tables)"
    copy = "__amd_rocclr_copyBuffer"
    _write_csv(str(prof / "trace" / "eq_kernel_stats.csv"),
               [{"Name": scale, "Calls": 48, "AverageNs": 380000, "TotalDurationNs": 48 * 380000,
                 "Percentage": 20.0}])
    mib = 256 * 1024  # KiB
    fetch = [{"Kernel_Name": copy, "Grid_Size": 262144, "Counter_Value": mib / 2}]
    fetch += [{"Kernel_Name": scale, "Grid_Size": 3145728, "Counter_Value": v} for v in (380000, 382000)]
    fetch += [{"Kernel_Name": digit, "Grid_Size": 2949120, "Counter_Value": 144000}]
    write = [{"Kernel_Name": copy, "Grid_Size": 262144, "Counter_Value": mib}]
    write += [{"Kernel_Name": scale, "Grid_Size": 3145728, "Counter_Value": 368000}]
    write += [{"Kernel_Name": digit, "Grid_Size": 2949120, "Counter_Value": 737000}]
    _write_csv(str(prof / "fetch" / "eq_counter_collection.csv"), fetch)
    _write_csv(str(prof / "write" / "eq_counter_collection.csv"), write)
    out = tmp_path / "out"
    bench.summarize_profiles(str(prof), str(out))
    t = json.load(open(out / "traffic.json"))
    assert t["calibration"]["factors"] == {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0}
    assert t["bytes_per_launch"]["scale"] == pytest.approx((381000 * 2 + 368000) * 1024)
    assert t["bytes_per_launch"]["ntt_digit"] == pytest.approx((144000 * 2 + 737000) * 1024)
    md = (out / "eq_mask_2p20_rows_kernels.md").read_text()
    assert "k_scale<15, true, 3>" in md and "--streams 1" in md
