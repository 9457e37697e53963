"""Build-level guards that need no GPU: every sample-aware kernel instance
(single-system, exact pass, batched, Pauli) keeps all values in registers.
The library also refuses such a build at run time (hipFuncGetAttributes);
this test catches a spilling build before it reaches a GPU.  The FP64
attentions and products are held to four waves per SIMD without spills."""
import os
import re
import subprocess

import pytest

from paper_2306_16705_amd import build as hip_build

KERNELS = re.compile(r"k_eloc_sa|k_eloc_pauli")


def _resource_usage(src, field="ScratchSize"):
    cmd = [hip_build.hipcc(), f"--offload-arch={hip_build.ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
           "--cuda-device-only", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", f"-I{hip_build.INCLUDE}", f"-I{hip_build.CSRC}",
           "-Rpass-analysis=kernel-resource-usage", os.path.join(hip_build.CSRC, src), "-o", os.devnull]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    usage, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"remark:\s+" + re.escape(field) + r" \[[^]]*\]: (\d+)", line)
        if m and name:
            usage[name] = int(m.group(1))
    return usage


@pytest.mark.parametrize("src", ["eloc_sa.hip", "pauli.hip"])
def test_sample_aware_kernels_do_not_spill(src):
    usage = _resource_usage(src)
    hot = {k: v for k, v in usage.items() if KERNELS.search(k)}
    assert hot, f"no sample-aware kernel found in {src}"
    spilled = {k: v for k, v in hot.items() if v != 0}
    assert not spilled, f"kernels with private-memory spills: {spilled}"
    if src == "eloc_sa.hip":
        names = " ".join(hot)
        for part in ("k_eloc_sa_exact", "k_eloc_sa_batch", "k_eloc_saI"):
            assert part in names, part


def test_fp64_list_kernels_run_four_waves_per_simd_without_spills():
    """Both attentions (whole sequence, list) and every FP64 product
    instance (plain, residual, LayerNorm-staged, QKV)."""
    scratch = _resource_usage("model_f64.hip")
    occ = _resource_usage("model_f64.hip", "Occupancy")
    names = [k for k in scratch if re.search(r"k64x?_attention|k64_gemm", k)]
    assert any("k64x_attention" in k for k in names), names
    assert any("k64_attention" in k for k in names), names
    assert sum("k64_gemm_res" in k for k in names) >= 2, names
    assert sum("k64_gemmI" in k for k in names) >= 5, names
    for k in names:
        assert scratch[k] == 0, k
        assert occ[k] >= 4, (k, occ[k])
