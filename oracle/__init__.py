"""Plain FP64 CPU oracle for the CUBE particle-mesh step (Yu, Pen & Wang, arXiv:1712.06121).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link this
package: only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use it. It shares no code with the HIP path (no kernels, headers, tables or constant
generators); the only things both sides consume are the seeded inputs produced by the
top-level ``synth`` module, which holds none of the method's arithmetic.

Modules
-------
cosmology   E(a), linear growth D(a) and f(a), kick/drift integrals, BBKS P(k), sigma_8
            normalisation, the linear velocity dispersion of Eq. (vdisp)/(vdelta).
philox      Philox4x32-10 counter-based generator and Box-Muller white noise (the random
            numbers the initial-condition generator draws), from its published definition.
ic          Zel'dovich initial conditions (Sec. 2.3.2, Fig. ic) on uncompressed particles.
pm          Plain FP64 particle-mesh code: CIC deposit, Poisson solve, 4-point gradient,
            CIC interpolation, DKD leapfrog (Sec. 2.3.3, Figs. code/update_xp/update_vp).
codec       FP64 reference of the storage formats: Eqs. (chi), (x), (nu), (v); cell counts
            and cell-ordered storage (Sec. 2.1, 2.2).
twin        FP32 step-by-step reference of the compressed step (load-encode, integer CIC,
            move from a given potential, per-cell moments, counting-sort order): the part
            the GPU must reproduce bit-exactly from identical inputs.
power       Auto and cross power spectra, Eqs. (cps), (ccc) and Delta^2(k) (Sec. 3).
displacement  Offsets of the same particle between two runs, Eq. (offset) (Sec. 3).
ewald       Periodic direct-sum (Ewald) forces for a handful of particles.
zeldovich   Exact 1-D Zel'dovich plane wave before shell crossing.
memory      Memory model of Sec. 2.4, Eqs. (npmax)-(Mp_fine) and Table t.memory.

Parity status of every function is listed in each module's header.
"""
