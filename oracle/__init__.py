"""TEST INFRASTRUCTURE ONLY: the plain FP64 CPU oracle of the track finding
and fitting path.  Imported only by the tests, the smoke check and the
benchmark's CPU-baseline leg."""
