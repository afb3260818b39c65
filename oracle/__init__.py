"""Reference oracle (test infrastructure only): plain FP64 CPU evaluation of
the likelihood the GPU library computes.  Imported only by tests, the smoke
check and the benchmark's CPU-baseline leg."""
