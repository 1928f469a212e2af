"""The measurement library's mqh_peak_probe (include/mqh_peak.h) on the GPU: each reference kernel
reports a positive rate within a plausible band of the MI355X spec peak it
measures (a copy or a read of 1-2 GiB, beyond the 256 MB last-level cache,
reaches at most the 8 TB/s HBM figure; FP32 FMA at most
157.3 TFLOP/s, two unpacked instructions per issue cycle; FP64 FMA and FP64
matrix cores at most 78.6 TFLOP/s).  The bands only catch a broken probe (wrong work count,
a kernel optimised away): the rates themselves are measurements."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mq():
    from paper_2511_09798_amd import peak

    return peak


@pytest.mark.parametrize("kind,size,lo,hi", [
    ("MQH_PEAK_COPY", 1 << 30, 1e12, 8.0e12),
    ("MQH_PEAK_READ", 1 << 31, 1e12, 8.0e12),
    ("MQH_PEAK_FMA_F32", 2048, 2e13, 157.4e12),
    ("MQH_PEAK_FMA_F64", 2048, 2e13, 78.7e12),
    ("MQH_PEAK_MFMA_F64", 2048, 2e13, 78.7e12),
])
def test_peak_probe_rates(mq, kind, size, lo, hi):
    say("peak probe", kind, size)
    rate = mq.mqh_peak_probe(getattr(mq, kind), size, reps=3)
    say("rate", rate)
    assert lo <= rate <= hi
