"""Coefficients of the short polynomials used by the fused loss kernel (loss.hip).

    python paper_2409_10876_amd/csrc/gen_poly.py

Each is a least-squares fit in the minimax sense (iteratively reweighted on a dense grid) of an odd or
even polynomial to the function on the reduced range the kernel uses, in float64; printed as C float
literals with the maximum absolute error on the range:

* atan(x) = x * P(x^2) on 0 <= x <= 1 (the kernel reduces atan2 to this range by swapping and reflecting);
* asin(x) = x * Q(x^2) on 0 <= x <= 1/2 (larger arguments use asin(x) = pi/2 - 2 asin(sqrt((1 - x) / 2)));
* sin(2 pi f) = f * S(f^2) and cos(2 pi f) = C(f^2) on |f| <= 1/8 revolution (the kernel reduces a phase in
  revolutions to this range and rotates by whole quarter turns).
"""
import numpy as np


def fit(fn, basis, lo, hi, iters=60):
    x = np.cos(np.linspace(0, np.pi, 4001)) * (hi - lo) / 2 + (hi + lo) / 2
    A = np.stack([b(x) for b in basis], -1)
    y = fn(x)
    w = np.ones_like(x)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(A * w[:, None], y * w, rcond=None)
        e = np.abs(A @ c - y)
        w *= (e / e.max() + 1e-3) ** 0.5
        w /= w.max()
    xs = np.linspace(lo, hi, 200001)
    err = np.abs(np.stack([b(xs) for b in basis], -1) @ c - fn(xs)).max()
    return c, err


def main():
    odd = lambda k: (lambda x: x ** (2 * k + 1))  # noqa: E731
    even = lambda k: (lambda x: x ** (2 * k))  # noqa: E731
    out = {}
    out["atan"] = fit(np.arctan, [odd(k) for k in range(8)], 0.0, 1.0)
    out["asin"] = fit(np.arcsin, [odd(k) for k in range(5)], 0.0, 0.5)
    out["sin2pi"] = fit(lambda f: np.sin(2 * np.pi * f), [odd(k) for k in range(4)], -0.125, 0.125)
    out["cos2pi"] = fit(lambda f: np.cos(2 * np.pi * f), [even(k) for k in range(5)], -0.125, 0.125)
    for name, (c, err) in out.items():
        lits = ", ".join(f"{float(np.float32(v))!r}f" for v in c)
        print(f"// {name}: max abs error {err:.2e} (float64)\nconstexpr float k_{name}[{len(c)}] = {{{lits}}};")


if __name__ == "__main__":
    main()
