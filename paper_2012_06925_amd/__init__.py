"""BLDTT compute phase on MI355X (gfx950): HIP kernels + C++ host engine behind a C ABI.

    from paper_2012_06925_amd import api
    plan = api.Plan(None, (x, y, z, q), kernel="coulomb", theta=0.7, degree=6, leaf=500)
    phi = plan.compute()

`inputs` holds the seeded synthetic particle generators; `build` compiles
libbldtt.so in-tree.  Importing the package loads nothing; `api` loads the
library and fails loudly when it has not been built.
"""
