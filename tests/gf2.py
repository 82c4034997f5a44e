"""GF(2) helpers for the oracle pins: Berlekamp-Massey and polynomial order.

Polynomials are Python ints, bit i = coefficient of x^i.  Nothing here is
shared with the oracle or the library.
"""
import sympy


def berlekamp_massey(bits):
    """Shortest LFSR of a GF(2) sequence.  Returns (L, C) with
    C = 1 + c1 x + ... + cL x^L such that s_n = sum_i c_i s_{n-i}."""
    Cp, Bp = 1, 1
    L, m = 0, 1
    for n, s in enumerate(bits):
        d = s
        for i in range(1, L + 1):
            d ^= ((Cp >> i) & 1) & bits[n - i]
        if d == 0:
            m += 1
        elif 2 * L <= n:
            T = Cp
            Cp ^= Bp << m
            L, Bp, m = n + 1 - L, T, 1
        else:
            Cp ^= Bp << m
            m += 1
    return L, Cp


def reciprocal(poly, deg):
    r = 0
    for i in range(deg + 1):
        if (poly >> i) & 1:
            r |= 1 << (deg - i)
    return r


def pmod(a, m):
    dm = m.bit_length() - 1
    while a and a.bit_length() - 1 >= dm:
        a ^= m << (a.bit_length() - 1 - dm)
    return a


def pmulmod(a, b, m):
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a.bit_length() - 1 >= m.bit_length() - 1:
            a = pmod(a, m)
    return pmod(r, m)


def ppowmod_x(e, m):
    """x^e mod m."""
    result, base = 1, pmod(2, m)
    while e:
        if e & 1:
            result = pmulmod(result, base, m)
        base = pmulmod(base, base, m)
        e >>= 1
    return result


def is_primitive(poly):
    """True iff poly (degree d, constant term 1) is primitive over GF(2):
    x has multiplicative order exactly 2^d - 1 modulo poly."""
    d = poly.bit_length() - 1
    if d < 1 or not (poly & 1):
        return False
    order = (1 << d) - 1
    if ppowmod_x(order, poly) != 1:
        return False
    for q in sympy.factorint(order):
        if ppowmod_x(order // q, poly) == 1:
            return False
    return True
