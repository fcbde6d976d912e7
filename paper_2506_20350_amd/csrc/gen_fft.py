#!/usr/bin/env python3
"""Generate straight-line in-register DFT codelets for every length 1..NMAX.

Output: a header with, for each length n and direction s (-1 forward,
+1 inverse, unnormalised):

    template<typename C> struct Fft<C, n, s> {
        static void run(C* v);   // v[k] <- sum_j v[j] exp(s 2 pi i jk / n)
        static void tw2(C* v);   // v[j] <- v[j] * exp(s 2 pi i j / (2n))
    };

Lengths with coprime factors use the prime-factor (Good-Thomas) algorithm,
which needs no twiddle factors (30 = 2 x 15 = 2 x 3 x 5); prime powers use
mixed-radix decimation in time (radix 4 first, then the prime); prime lengths
use the direct DFT written with the conjugate-pair symmetry x_j +- x_{p-j}.  Twiddles are literal double
constants (17 significant digits) cast to the element type, so single and
double precision codelets share one source.  The arrays are indexed only with
constants, which keeps them in registers after inlining.
"""
import math
import sys

NMAX = 64


class Emit:
    def __init__(self):
        self.lines = []
        self.n = 0

    def tmp(self, expr):
        name = f"t{self.n}"
        self.n += 1
        self.lines.append(f"const C {name} = {expr};")
        return name


def lit(x):
    if abs(x) < 1e-300:
        x = 0.0
    return f"R({x!r})"


def add(e, a, b):
    if a is None:
        return b
    if b is None:
        return a
    return e.tmp(f"cadd({a}, {b})")


def sub(e, a, b):
    if b is None:
        return a
    if a is None:
        return e.tmp(f"cneg({b})")
    return e.tmp(f"csub({a}, {b})")


def mul_i(e, a, s):
    """a * (s i), s = +-1."""
    if a is None:
        return None
    return e.tmp(f"cmuli({a})" if s > 0 else f"cmulni({a})")


def twiddle(e, a, num, den, s):
    """a * exp(s 2 pi i num / den)."""
    if a is None:
        return None
    num %= den
    if num == 0:
        return a
    if (4 * num) % den == 0:
        q = (4 * num) // den          # quarter turns
        if q == 2:
            return e.tmp(f"cneg({a})")
        return mul_i(e, a, s if q == 1 else -s)
    ang = 2.0 * math.pi * num / den
    c, si = math.cos(ang), s * math.sin(ang)
    return e.tmp(f"cmulc({a}, {lit(c)}, {lit(si)})")


def small_dft(e, x, s):
    n = len(x)
    if n == 1:
        return list(x)
    if n == 2:
        return [add(e, x[0], x[1]), sub(e, x[0], x[1])]
    if n == 4:
        t0, t1 = add(e, x[0], x[2]), sub(e, x[0], x[2])
        t2 = add(e, x[1], x[3])
        t3 = mul_i(e, sub(e, x[1], x[3]), s)
        return [add(e, t0, t2), add(e, t1, t3), sub(e, t0, t2), sub(e, t1, t3)]
    # odd length: conjugate-pair form
    h = (n - 1) // 2
    a = [None] + [add(e, x[j], x[n - j]) for j in range(1, h + 1)]
    d = [None] + [sub(e, x[j], x[n - j]) for j in range(1, h + 1)]
    out = [None] * n
    acc = x[0]
    for j in range(1, h + 1):
        acc = add(e, acc, a[j])
    out[0] = acc
    for k in range(1, h + 1):
        A = x[0]
        B = None
        for j in range(1, h + 1):
            jk = (j * k) % n
            c = math.cos(2.0 * math.pi * jk / n)
            sn = math.sin(2.0 * math.pi * jk / n)
            if a[j] is not None:
                A = e.tmp(f"cfmar({a[j]}, {lit(c)}, {A})") if A is not None else e.tmp(f"cscale({a[j]}, {lit(c)})")
            if d[j] is not None:
                B = e.tmp(f"cfmar({d[j]}, {lit(sn)}, {B})") if B is not None else e.tmp(f"cscale({d[j]}, {lit(sn)})")
        iB = mul_i(e, B, s)
        out[k] = add(e, A, iB)
        out[n - k] = sub(e, A, iB)
    return out


def smallest_factor(n):
    if n % 4 == 0 and n > 4:
        return 4
    for p in range(2, n + 1):
        if n % p == 0:
            return p
    return n


def coprime_split(n):
    """n = a * b with gcd(a, b) = 1 and a, b > 1 (a the power of the smallest prime), or None."""
    p = next(q for q in range(2, n + 1) if n % q == 0)
    a, m = 1, n
    while m % p == 0:
        a, m = a * p, m // p
    return (a, m) if m > 1 else None


def fft(e, x, s):
    n = len(x)
    if n <= 2 or n == 4:
        return small_dft(e, x, s)
    sp = coprime_split(n)
    if sp:
        # Good-Thomas prime-factor algorithm: with the input map n = (b n1 + a n2) mod N and
        # the output map k = (k1 b (b^-1 mod a) + k2 a (a^-1 mod b)) mod N, the N-point DFT is an
        # a x b two-dimensional DFT without twiddle factors.
        a, b = sp
        cols = [fft(e, [x[(b * n1 + a * n2) % n] for n1 in range(a)], s) for n2 in range(b)]
        ainv, binv = pow(a, -1, b), pow(b, -1, a)
        out = [None] * n
        for k1 in range(a):
            y = fft(e, [cols[n2][k1] for n2 in range(b)], s)
            for k2 in range(b):
                out[(k1 * b * binv + k2 * a * ainv) % n] = y[k2]
        return out
    r = smallest_factor(n)
    if r == n:
        return small_dft(e, x, s)
    m = n // r
    subs = [fft(e, x[j::r], s) for j in range(r)]
    out = [None] * n
    for k2 in range(m):
        col = [twiddle(e, subs[j][k2], j * k2, n, s) for j in range(r)]
        y = small_dft(e, col, s)
        for k1 in range(r):
            out[k2 + m * k1] = y[k1]
    return out


def codelet(n, s):
    e = Emit()
    x = []
    for j in range(n):
        x.append(e.tmp(f"v[{j}]"))
    y = fft(e, x, s)
    body = list(e.lines)
    for k in range(n):
        body.append(f"v[{k}] = {y[k] if y[k] is not None else 'czero<C>()'};")
    e2 = Emit()
    tw = []
    for j in range(n):
        t = twiddle(e2, f"v[{j}]", j * s if s > 0 else -j, 2 * n, 1)
        tw.append((j, t))
    body2 = list(e2.lines) + [f"v[{j}] = {t};" for j, t in tw if t != f"v[{j}]"]
    ind = "        "
    return (f"template<typename C> struct Fft<C, {n}, {s}> {{\n"
            f"    typedef typename CTraits<C>::real R;\n"
            f"    static __device__ __forceinline__ void run(C* v) {{\n"
            + "".join(ind + l + "\n" for l in body) +
            f"    }}\n"
            f"    static __device__ __forceinline__ void tw2(C* v) {{\n"
            + "".join(ind + l + "\n" for l in body2) +
            f"    }}\n}};\n")


def main(path, nmax=NMAX):
    parts = ["// Generated by gen_fft.py: in-register DFT codelets. Do not edit.\n",
             "#pragma once\n#include \"common.h\"\n\n",
             "template<typename C, int N, int S> struct Fft;\n\n"]
    for n in range(1, nmax + 1):
        for s in (-1, 1):
            parts.append(codelet(n, s))
    with open(path, "w") as f:
        f.write("".join(parts))


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else NMAX)
