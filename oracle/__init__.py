"""CPU oracle for the GraphVine operations.

TEST INFRASTRUCTURE ONLY: the plain ordered-set definition the GPU structure
is checked against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library.
"""
