"""Generate the 10-node, degree-5, fully symmetric triangle rule (run: python -m workloads.gen_rule10).

The paper's Vioreanu--Rokhlin rules (Section 3, quadrature paragraph) are tabulated in a
reference that is not reproduced here, so the build uses its own rule with the
properties the method needs: n_q = 10 strictly interior nodes (p = 3 interpolation,
n_q = (p+1)(p+2)/2), positive weights and exactness for all polynomials of total degree
<= 5 (d_ex = 5 > p).

Orbit structure 1 + 3 + 6 in barycentric coordinates:
  centroid (1/3, 1/3, 1/3) with weight w0,
  the 3 permutations of (a, a, 1-2a) with weight w1,
  the 6 permutations of (b, c, 1-b-c) with weight w2.
Five symmetric moment conditions leave a one-parameter family.  Its P3 Lebesgue
constant decreases monotonically as the nodes approach the vertices, so it has no
interior minimiser; the member used here is the "equal-margin" one, b = a, where every
non-centroid node has the same smallest barycentric coordinate (this maximises that
smallest coordinate over the family).  The five remaining unknowns are found by Newton
iteration at 40 significant digits and printed as Python source.
"""
import itertools

import mpmath as mp

mp.mp.dps = 40


def _moments(w0, w1, w2, a, c):
    b = a
    pts = [((mp.mpf(1) / 3,) * 3, w0)]
    pts += [(p, w1) for p in set(itertools.permutations((a, a, 1 - 2 * a)))]
    pts += [(p, w2) for p in set(itertools.permutations((b, c, 1 - b - c)))]
    # symmetric invariants of degree 0, 2, 3, 4, 5 in barycentric coordinates
    inv = [lambda l: 1,
           lambda l: l[0] ** 2 + l[1] ** 2 + l[2] ** 2,
           lambda l: l[0] * l[1] * l[2],
           lambda l: l[0] ** 4 + l[1] ** 4 + l[2] ** 4,
           lambda l: l[0] * l[1] * l[2] * (l[0] ** 2 + l[1] ** 2 + l[2] ** 2)]
    # exact integrals over the reference triangle of area 1/2:
    #   int l1^i l2^j l3^k = i! j! k! / (i+j+k+2)!
    exact = [mp.mpf(1) / 2, mp.mpf(1) / 4, mp.mpf(1) / 120, mp.mpf(1) / 10, mp.mpf(1) / 280]
    return [sum(wt * f(p) for p, wt in pts) - e for f, e in zip(inv, exact)]


def solve():
    guess = (mp.mpf('0.0995'), mp.mpf('0.0302'), mp.mpf('0.0516'), mp.mpf('0.0711'), mp.mpf('0.314'))
    sol = mp.findroot(lambda *v: _moments(*v), guess, tol=mp.mpf(10) ** -36)
    return [sol[i] for i in range(5)]


if __name__ == '__main__':
    w0, w1, w2, a, c = solve()
    print(f"W0 = {mp.nstr(w0, 30)}")
    print(f"W1 = {mp.nstr(w1, 30)}")
    print(f"W2 = {mp.nstr(w2, 30)}")
    print(f"A = {mp.nstr(a, 30)}")
    print(f"C = {mp.nstr(c, 30)}")
