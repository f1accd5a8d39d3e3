"""CPU oracle for the DovetailSort hot path -- TEST INFRASTRUCTURE ONLY.

Nothing in the product (the HIP library and its Python binding) may import,
call, link or execute anything in this package.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg use it.  It shares no code with the
GPU path: the only thing both sides consume is the seeded input generators in
``workloads``, which hold none of the method's arithmetic.

Modules
-------
``sort``        the plain definition of a stable sort (Section 2.3: records in
                non-decreasing key order, equal keys in input order), a
                brute-force rank formula, segmented sort and invariant checks.
``rng``         the splitmix64 output function and the counter-based sample
                index generator the method's sampling step draws from.
``dtsort_ref``  the method's steps written in the paper's order (Alg. 2 and
                Sections 3.1-3.5, plus the overflow bucket of Section 5):
                planning and sampling, GetBucketId, the stable counting sort
                (Appendix B), the dovetail merge (Alg. 3) and the recursion.
``psort``       the same definition on all host cores (C++, libstdc++'s parallel
                stable sort; built by ``build()``): the benchmark's multicore
                CPU baseline.
``mlp``         the learned partitioner's 1-64-64-1 CDF model in float64:
                forward, backward, Adam, splitter inversion, balance error.
                Not in the paper; parity of the training trajectory is
                unpinned beyond tolerance.
"""
