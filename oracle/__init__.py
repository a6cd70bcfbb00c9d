"""CPU oracles for the NARVis hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the GPU library and does not
import it: inputs are handed in as plain arrays.
"""
