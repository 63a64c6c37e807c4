"""CPU reference oracle for the compact-Helmholtz / EigT-GMRES method (complex128, numpy + scipy).

TEST INFRASTRUCTURE ONLY. Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py`
may import or execute anything in this package. The product (the HIP library and its Python binding) never
calls it, and this package never imports the product: the two share no code. The only shared module is
`synth`, which samples seeded input fields and holds none of the method's arithmetic.

Every function cites the passage of the paper (arXiv 2602.07711) it follows by section, equation, algorithm or
table. Readings of passages that are ambiguous are listed in the module docstrings where they are used.
"""
from . import operators, precond, krylov  # noqa: F401
