"""The measurement library's mqh_peak_probe (include/mqh_peak.h) on the GPU: each reference kernel
reports a positive rate within a plausible band of the MI355X spec peak it
measures (a copy or a read of 1-2 GiB, beyond the 256 MB last-level cache,
reaches at most the 8 TB/s HBM figure; FP32 FMA at most
157.3 TFLOP/s, two unpacked instructions per issue cycle; FP64 FMA and FP64
matrix cores at most 78.6 TFLOP/s; the transcendental unit at most a quarter of the FP32 lane
rate; bf16 matrix cores at most 2.5 PFLOP/s).  The bands only catch a broken probe (wrong work count,
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
    # one transcendental lane operation per lane per four cycles at most (16 lanes of a SIMD per cycle)
    ("MQH_PEAK_RSQ_F32", 1024, 1e12, 39.4e12),
    ("MQH_PEAK_RSQ_FMA_F32", 512, 5e11, 39.4e12),
    # bf16 matrix cores: 2.5 PFLOP/s dense
    ("MQH_PEAK_MFMA_BF16", 2048, 1e14, 2.52e15),
])
def test_peak_probe_rates(mq, kind, size, lo, hi):
    say("peak probe", kind, size)
    rate = mq.mqh_peak_probe(getattr(mq, kind), size, reps=3)
    say("rate", rate)
    assert lo <= rate <= hi
