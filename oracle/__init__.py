"""FP64 CPU oracle for the state-vector simulator.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg may import it; the simulator never does."""
