"""Parity bars of the GPU tests, with where they come from.

FP64: the HIP path and the FP64 oracle evaluate the same estimator in the
same precision, differing only in the order of rounding: per-probe values
within 1e-10 relative (to the mean |h_j|), moments within 1e-10 ||g||^2.

Reduced precision, against the FP64 oracle on the same stored input:
* FP32 products (FP64 reductions): each product carries a relative error of
  order sqrt(K) u_32 (u_32 = 6e-8, K the inner dimension) and the m steps add
  them.  Measured per-probe errors: 1e-8 .. 4e-7 (up to n = 10^7 banded and
  n = 8192 dense).  Bar 1e-5.
* BF16x3 (three bf16 products with FP32 accumulation): every step re-splits
  V_{k+1} into bf16 hi + lo, which keeps about 17 significant bits, so each
  step adds a relative error of order 2^-17 = 7.6e-6 per entry (the split of
  R the same once); over m steps these add like a random walk, sqrt(m) 2^-17
  = 5.4e-5 at m = 50.  Measured per-probe errors: 3e-7 .. 4e-6.  Bar 5e-5.
A loss of accuracy of an order or two (an FP32 reduction of the per-probe
dots, a missing lo term of the split) fails these bars.
"""
TOL64 = 1e-10
TOL_F32 = 1e-5
TOL_BF16X3 = 5e-5


def tol_for(precision: str) -> float:
    return {"f64": TOL64, "f32": TOL_F32, "bf16x3": TOL_BF16X3}[precision]
