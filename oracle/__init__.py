"""FP64 CPU oracle of the LEAD decoder -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The decoder library never does, and shares no source
with it."""
