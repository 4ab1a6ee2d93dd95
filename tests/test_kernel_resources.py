"""Register and scratch use of the hot-path kernels, read from the compiler's resource report for
gfx950 (no GPU needed). A kernel on the hot path that spills to scratch memory loses much of its
speed without any change in its results, so the parity tests cannot see it; this test can.
Vector registers may not spill at all and no kernel may use scratch memory; scalar registers may
spill only into lanes of vector registers (scratch size 0), which costs one lane move each."""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_17556_amd", "csrc")

# kernel (demangled-name fragment as it appears in the mangled symbol) -> source file
HOT = {
    "gram_kernel_fp8": "gram.hip",
    "gram_kernel_split": "gram.hip",
    "gram_reduce_kernel": "gram.hip",
    "refine_pass_kernelILi32": "gemv.hip",
    "refine_pass_kernelILi16": "gemv.hip",
    "refine_pass_kernelILi8": "gemv.hip",
    "refine_line_kernelILi32ELb1": "gemv.hip",
    "refine_line_kernelILi32ELb0": "gemv.hip",
    "refine_line_kernelILi16ELb0": "gemv.hip",
    "refine_line_kernelILi8ELb0": "gemv.hip",
    "rowpass_prep_kernelILb1ELi3": "gemv.hip",
    "colpass_kernelILi0": "gemv.hip",
    "rowpass_multi_t_kernel": "multi.hip",
    "rowpass_multi_tm_kernel": "multi.hip",
    "colpass_multi_mfma_kernel": "multi.hip",
    "potf2_kernel": "potrf.hip",
    "update_kernel": "potrf.hip",
    "trsm_kernel": "potrf.hip",
    "fp8_apply_kernel": "apply8.hip",
    "final_decide_kernel": "apply8.hip",
    "fwd_step2_kernel": "trsv.hip",
    "bwd_step2_kernel": "trsv.hip",
}


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def _report(src):
    cmd = [_hipcc(), "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only", "-c", "-x", "hip",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", os.path.join(CSRC, src), "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    kernels, cur = {}, None
    for line in out.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = kernels.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z /\[\]]+?): (\S+) \[-Rpass", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = m.group(2)
    return kernels


@pytest.fixture(scope="module")
def reports():
    if _hipcc() is None:
        pytest.skip("hipcc not available")
    srcs = sorted(set(HOT.values()))
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        return dict(zip(srcs, ex.map(_report, srcs)))


@pytest.mark.parametrize("frag", sorted(HOT))
def test_hot_kernel_does_not_spill(reports, frag):
    rep = reports[HOT[frag]]
    hits = {name: r for name, r in rep.items() if frag in name}
    assert hits, f"no kernel matching {frag} in {HOT[frag]}"
    for name, r in hits.items():
        assert r.get("ScratchSize [bytes/lane]") == "0", (name, r)
        assert r.get("VGPRs Spill") == "0", (name, r)
