"""Write the FP64 oracle's result on the full reduced-precision workload
(512^3, SO8, 1000 steps; helpers.c4_case with every 4th receiver of each line)
to c4_reference.npz, for the GPU tests that compare each storage format with it.

Only the oracle computes here (the inputs come from the seeded generators). The
stored values:
  traces   [1000][256] float32  oracle traces (rounded once from FP64)
  sample   [64][64][64] float32 u^1000 on the sub-lattice k, j, i = 4, 12, ..., 508
  norm_field, norm_sample, max_sample   FP64 norms of u^1000 and of the sample
  meta     JSON text: the case and the sample definition

The oracle needs about 10 GB of RAM and 10-20 minutes on 8 cores:
    python tests/golden/make_c4_reference.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))            # tests/ (helpers)
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))  # repository root

import oracle  # noqa: E402
from helpers import c4_case  # noqa: E402

OUT = os.path.join(HERE, "c4_reference.npz")
REC_STRIDE = 4
SAMPLE = (4, 8)  # offset, stride of the field sub-lattice on every axis


def main():
    case = c4_case(rec_stride=REC_STRIDE)
    print("oracle C4: %s SO%d nt=%d dt=%.9g, %d receivers, threads %d"
          % (case.n, case.so, case.nt, case.dt, len(case.rec), oracle.num_threads()), flush=True)
    t0 = time.perf_counter()
    rec, uf, _ = case.oracle_forward()
    el = time.perf_counter() - t0
    o, s = SAMPLE
    smp = uf[o::s, o::s, o::s]
    meta = {"case": "c4_case(n=(512,512,512), nt=1000, nbl=40, rec_stride=%d)" % REC_STRIDE,
            "so": case.so, "nt": case.nt, "dt": case.dt, "nrec": int(len(case.rec)),
            "sample_offset": o, "sample_stride": s, "oracle_seconds": round(el, 1),
            "oracle_threads": oracle.num_threads()}
    np.savez_compressed(OUT, traces=rec.astype(np.float32), sample=smp.astype(np.float32),
                        norm_field=np.float64(np.linalg.norm(uf)),
                        norm_sample=np.float64(np.linalg.norm(smp)),
                        max_sample=np.float64(np.abs(smp).max()),
                        norm_traces=np.float64(np.linalg.norm(rec)),
                        meta=np.array(json.dumps(meta)))
    print("wrote %s (%.1f s of oracle): |u| %.6e, |sample| %.6e, |traces| %.6e"
          % (OUT, el, np.linalg.norm(uf), np.linalg.norm(smp), np.linalg.norm(rec)), flush=True)


if __name__ == "__main__":
    main()
