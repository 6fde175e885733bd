"""Seeded, synthetic problem inputs shared by the oracle, the tests and the benchmark.

Nothing in this package computes any part of the method (no Green's function, no
correction, no solver).  It produces only what a user of the solver would hand it:
quadrature nodes and weights on a curved triangular mesh, the subdomain of every
element, the analytic boundary curves, the contrast at the nodes, incident plane
waves and seeded random vectors.
"""
