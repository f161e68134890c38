"""CPU oracle for the QuadBox rasterizer hot path -- test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU path.
"""
