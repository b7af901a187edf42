"""FP64 CPU oracle of the adaptive-precision (AP) energy and force path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import or call anything in this package;
the product path (the HIP library and its Python binding) never does.  The
oracle shares no code with the HIP library: no kernels, headers, helpers or
table/constant generators.  The only thing both consume is the seeded input
generator ``paper_2505_12958_amd.workloads`` (inputs only, no method
arithmetic).

Everything is plain, slow and written from the definitions, in float64:

* ``geometry``  - canonical minimum-image displacement, brute-force and
  k-d-tree-candidate neighbour lists (bit-exact inclusion rule);
* ``tables``    - evaluation of the uniform-knot piecewise-cubic EAM tables;
* ``eam_analytic`` - the paper's W EAM in closed form (ZBL core, quintic
  bridge, knot sums, clamped density, square-root embedding);
* ``eam``       - EAM per-atom energy E_i = xi(sum_j zeta) + 1/2 sum_j Phi
  (paper, equation for E_i^EAM) and its gradient w.r.t. each bond vector;
* ``ylm``       - real orthonormal spherical harmonics and their gradients;
* ``cg``        - complex Clebsch-Gordan coefficients (Racah's closed form)
  and their real-harmonic transform;
* ``ace``       - ACE atomic basis A_nlm, product basis B_v, the embedding
  E_i = phi^(1) + sqrt(|phi^(2)| + 1e-6) (paper, ACE energy equation with
  the guard at phi^(2)=0) and the chain-rule bond gradients;
* ``switching`` - the per-atom switching parameter lambda_i (ACE weight):
  geometric rules with their gradient, and the paper's CSP-driven dynamic
  switching with time averages and a transition zone;
* ``ap``        - the AP blend E = sum_i [lambda_i E_i^ACE + (1-lambda_i) E_i^EAM]
  (paper, equation E_i for the AP potential, with lambda = ACE weight),
  forces -dE/dr at fixed lambda (plus the grad-lambda term of a geometric
  rule), the virial, and the spherical indenter V_ind with its load P_ind;
* ``md``        - FP64 velocity-Verlet with fixed atoms and the Nose-Hoover
  layer of the nanoindentation protocol (and its conserved extended energy);
* ``indentation`` - depth, Hertzian load and its fit for E*, contact radius
  and hardness of a load curve.

Pins (tests marked "not gpu") tie each function to what the paper or the
mathematics fixes; see the test files for each pin.  The synthetic ACE model
itself has no published counterpart: its physics is parity unpinned (only
invariances, closed forms and finite differences pin the arithmetic).
"""
