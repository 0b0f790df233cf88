"""Derive the polynomial for 2^f, f in [-1/2, 1/2], used by the FP64 kernel exponential.

The FP64 kernels evaluate exp(-D^2/eps) as 2^q with q = -D^2 log2(e)/eps, split q = n + f with
n = rint(q) (so f = q - n is exact and |f| <= 1/2), and 2^q = ldexp(p(f), n).  p is a degree-10
near-minimax polynomial for 2^f on [-1/2, 1/2], obtained here by Chebyshev fitting in 50-digit
arithmetic and rounded to double; the script also reports the worst relative error of the rounded
polynomial (evaluated with Horner's rule in exact arithmetic) on a dense grid.

Run: python paper_1905_10587_amd/csrc/gen_exp2_poly.py   (prints the coefficients used in kmv_kernels.h)
"""
import mpmath as mp

mp.mp.dps = 50
DEG = 10


def main():
    f = lambda x: mp.power(2, x)  # noqa: E731
    poly, err = mp.chebyfit(f, [-0.5, 0.5], DEG + 1, error=True)
    coeffs = [float(c) for c in reversed(poly)]          # ascending powers, rounded to double
    worst = mp.mpf(0)
    for i in range(4001):
        x = mp.mpf(-0.5) + mp.mpf(i) / 4000
        acc = mp.mpf(0)
        for c in reversed(coeffs):
            acc = acc * x + mp.mpf(c)
        worst = max(worst, abs(acc / f(x) - 1))
    print(f"# degree {DEG}, fit error {mp.nstr(err, 3)}, worst relative error after rounding {mp.nstr(worst, 3)}")
    for k, c in enumerate(coeffs):
        print(f"c{k} = {c!r}  # {c.hex()}")


if __name__ == "__main__":
    main()
