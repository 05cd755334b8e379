"""Report of the operator GEMM tile plans and the device's measured ceilings.

    python -m paper_1312_1638_amd.gemm_sweep

Times every instantiated (row blocks, column strips) plan of the library's
matrix-core GEMM on the operator shapes of hex p=3 (16^3 and 48^3 elements)
and hex p=4 (48^3), FP64 and FP32, and prints the fastest and slowest plans
per shape; the set-up autotuner makes the same choice per mesh.
"""
import sys

SHAPES = [(1, 1), (1, 2), (1, 4), (2, 1), (2, 2), (2, 4), (3, 1), (3, 2), (3, 4), (4, 1),
          (4, 2), (4, 4), (6, 1), (6, 2), (6, 4), (8, 1), (8, 2), (12, 1), (12, 2)]
CASES = [("M0 p3", 96, 64, 0, 20480, 1), ("S3 p3", 192, 96, 64, 20480, 1),
         ("M5 p3", 96, 64, 0, 20480, 3), ("S8 p3", 64, 96, 192, 20480, 1),
         ("M0 p4 L", 150, 125, 0, 552960, 1), ("S8 p4 L", 125, 150, 375, 552960, 1),
         ("S3 p3 L", 192, 96, 64, 552960, 1)]


def main():
    from . import binding as B
    print("ceilings: HBM GB/s %.0f  FP64 MFMA TF %.1f  FP32 MFMA TF %.1f" % (
        B.measure_ceiling(0), B.measure_ceiling(1), B.measure_ceiling(2)), flush=True)
    for prec in ("fp64", "fp32"):
        for name, M, K1, K2, N, batch in CASES:
            MB = -(-M // 16)
            res = []
            for mbw, nc in SHAPES:
                wm = -(-MB // mbw)
                if mbw * (wm - 1) >= MB:
                    continue
                ms = B.bench_gemm(prec, M, K1, K2, N, (mbw, nc, wm), batch, 10)
                tf = 2.0 * M * (K1 + K2) * N * batch / (ms * 1e-3) / 1e12
                res.append((ms, mbw, nc, wm, tf))
            res.sort()
            print(prec, name, " ".join("[%d,%d,%d] %.1fus %.1fTF" % (m, n, w, ms * 1e3, tf)
                                       for ms, m, n, w, tf in res[:6]), flush=True)
            print("   worst", " ".join("[%d,%d,%d] %.1fus" % (m, n, w, ms * 1e3)
                                       for ms, m, n, w, tf in res[-3:]), flush=True)


if __name__ == "__main__":
    sys.exit(main())
