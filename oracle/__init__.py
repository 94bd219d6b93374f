"""Oracle for the dense Tucker / HOOI hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct CPU implementation of what the GPU path
computes, written from the paper (Chakaravarthy et al., "On Optimizing
Distributed Tucker Decomposition for Dense Tensors", arXiv 1707.05594):

* ``oracle.hooi``  -- FP64 NumPy HOOI: TTM (Sec. 2.1), naive per-mode TTM
  chain (Fig. 2 "HOOI Procedure"), leading singular vectors through the Gram
  matrix and an eigensolver (Sec. 5), HOSVD start, new core, error.
* ``oracle.plan``  -- TTM-tree cost model (Sec. 3.1), the optimal-tree
  dynamic program (Sec. 3.3, recurrence), chain and balanced trees (Sec. 3.2),
  and a brute-force enumerator of all trie-shaped TTM-trees (plain C,
  ``brute_plan.c``) used to pin the dynamic program.
* ``oracle.precision`` -- exact float64 models of the BF16 and split-BF16
  (bf16x3) TTM node: operand rounding to bfloat16 and the kept products.
* ``oracle.mlp`` -- float64 forward, chain-rule gradient and Adam step of the
  cost model used for learned tree selection.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The product path never calls it and shares no
code with it: the GPU library and this oracle are independent
implementations that meet only on the seeded inputs produced by ``synth``.
"""
