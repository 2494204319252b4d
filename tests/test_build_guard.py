"""The build's scratch-memory guard (paper_2301_13601_amd/build.py): it reads
the compiler's resource-usage remarks and names every kernel that uses
scratch memory."""
from paper_2301_13601_amd.build import spilled_kernels

REMARKS = """\
qnn.hip:158:1: remark: Function Name: _ZN3qnn6good_kernelEv [-Rpass-analysis=kernel-resource-usage]
qnn.hip:158:1: remark:     VGPRs: 112 [-Rpass-analysis=kernel-resource-usage]
qnn.hip:158:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
qnn.hip:250:1: remark: Function Name: _ZN3qnn7spilledEv [-Rpass-analysis=kernel-resource-usage]
qnn.hip:250:1: remark:     VGPRs: 256 [-Rpass-analysis=kernel-resource-usage]
qnn.hip:250:1: remark:     ScratchSize [bytes/lane]: 192 [-Rpass-analysis=kernel-resource-usage]
qnn.hip:300:1: remark: Function Name: _ZN3qnn5otherEv [-Rpass-analysis=kernel-resource-usage]
qnn.hip:300:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
"""


def test_spilled_kernels_names_only_kernels_with_scratch():
    assert spilled_kernels(REMARKS) == [("_ZN3qnn7spilledEv", 192)]


def test_spilled_kernels_empty_without_remarks():
    assert spilled_kernels("") == []
    assert spilled_kernels("warning: loop not unrolled\n") == []
