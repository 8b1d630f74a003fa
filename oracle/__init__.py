"""CPU oracle for syndrome-adaptive-gain min-sum decoding of GB QLDPC codes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the ``libsagms`` C-ABI
library, its Python binding, the kernels) imports, links or calls anything in
this package.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.

The oracle is a plain, slow, obviously checkable restatement of the method of
Cordova et al., "Syndrome Adaptive Gain Control for Min-Sum Decoding of
Quantum LDPC Codes" (arXiv 2605.10433), written in NumPy, FP64 unless a
function says otherwise.  It shares no code, tables or constants with the
HIP path.  Each module cites the section / equation / algorithm it follows.

Modules
  gf2       GF(2) linear algebra (rank, nullspace, rowspace membership)
  codes     generalized-bicycle codes, code dimension, logical basis
  philox    Philox4x32-10 counter-based generator (Salmon et al., SC'11)
  channel   depolarizing channel sampling, syndromes, bit packing, prior LLR
  decoders  MS / SMS / SAGMS / BP decoders (Alg. 1), FP64 and FP32 modes
  layered   the layered (check-serial) schedule of the min-sum family
  judge     logical-failure judge (rank test and logical-operator test)
  stats     Wilson interval and log-ratio interval of an FER ratio
  analysis  transfer functions, BP-matching ratio, op-count model

Parity status of each function is stated in its docstring.  Every function
here is pinned by a ``-m "not gpu"`` test against something other than
itself (closed forms, brute force, printed values of the paper, an
independent library); none is "parity unpinned".
"""
