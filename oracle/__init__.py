"""FP64 CPU oracle for the per-frame Gauss-Newton warp-field solve.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute anything in this package; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it. It shares no code with the HIP path.

It is a plain, slow, step-by-step reading of the paper (SurfelWarp, Gao and
Tedrake, RSS 2019):

* Sec. 3 (Preliminaries): node graph warp field, dual-quaternion blend of the
  nearest nodes (Eq. 1) and surfel deformation (Eq. 2);
* Sec. 5 (Depth Image Processing): vertex map by back-projection, normal map by
  central differences;
* Sec. 6.5 (Initialization): skinning of surfels to their nearest nodes;
* Sec. 7 (Non-Rigid Warp Field Estimation): index-map visibility, the total
  energy, the point-to-plane data term and the as-rigid-as-possible
  regulariser, minimised by Gauss-Newton;
* Sec. 8 (Implementation Details): build J^T J, then solve; at most 10
  Gauss-Newton iterations;
* Table 1: node sampling distance 2.5 cm, regulariser weight 5.

Floating point is FP64 throughout, except where a floating-point comparison
decides an integer (nearest-node order, pixel of a projection, index-map
winner, validity gates). Those decisions are taken in FP32 with one fixed
operation order (module `replica32`), the precision the GPU kernels decide in,
so that integer outputs can be compared bit for bit.

Modules:
  quat      quaternion and dual-quaternion algebra, SO(3) exponential
  skin      nearest-node skinning and the node graph
  depth     vertex and normal maps of a depth image
  warp      dual-quaternion blend, its application and its derivatives
  assoc     index map and projective correspondence
  terms     residuals, energies and Jacobians of both energy terms
  solve     normal equations, Cholesky / block-Jacobi PCG, node update, GN
  replica32 FP32 decision replica
"""
