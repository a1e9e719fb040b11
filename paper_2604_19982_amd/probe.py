"""Roofline calibration on the current device.

Runs the register-only FMA probes (scalar FP32, FP64) and one plain copy of
a known size (2 GiB: 1 GiB read + 1 GiB written); under rocprofv3 --pmc the
copy kernel's FETCH_SIZE / WRITE_SIZE give the scale of the HBM byte
counters.  Prints one JSON line.
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import paper_2604_19982_amd as pj  # noqa: E402

COPY_BYTES = 1 << 30


def main():
    c = pj.Context()
    out = {"fp32_fma_gflops": max(c.probe_fma(False) for _ in range(3)),
           "fp64_fma_gflops": max(c.probe_fma(True) for _ in range(2)),
           "copy_bytes": COPY_BYTES, "copy_gbps": c.probe_copy(COPY_BYTES)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
