"""Plain FP64 CPU oracle of the plane-strain LBM (arXiv 2301.00228).

Test infrastructure only: the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg use it to check and time the GPU library.  It
shares no code with the GPU library and the GPU library never imports it.
"""
