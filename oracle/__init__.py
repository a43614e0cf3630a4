"""FP64 CPU oracle of the G-REST update.  Test infrastructure: only the tests, the
smoke check and the benchmark's CPU-baseline leg use it."""
