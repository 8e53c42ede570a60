"""FP64 CPU oracle for qFlex-style random-circuit amplitudes.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check and
the CPU-baseline leg of the benchmark may import this package.  The product
path (the HIP library and its Python binding) never imports, calls or links it,
and this package imports nothing from the product path.  Inputs (circuit text,
plans, bitstrings) come from the `workloads` package, which holds no arithmetic
of the method.

Modules
    gates    gate matrices written from their definitions, own table
    parse    own parser of the circuit text format and plan dictionaries
    sv       direct state-vector evolution (paper Sec. II, first simulator
             class): the plain definition a(x) = <x| U |0...0>; and the state
             of one path of the sliced sum (Sec. III-A, III-C)
    tn       tensor-network route (paper Sec. II, tensor-network class, and
             Sec. III): time-first world-line tensors, sliced pairwise
             contraction in a given plan order, complex128 throughout
    grad     adjoint state-vector gradient of the amplitudes with respect to
             every gate's entries, and exact central finite differences
    metrics  norm-wise relative error and Porter-Thomas statistics

Every public function in these modules is pinned by a CPU test against a
closed form, an invariant, a brute-force product or a library routine; none of
them is "parity unpinned".
"""
