"""Oracle for the Brouwer-Zimmermann minimum-distance path (test infrastructure).

A plain CPU implementation in mod-p integer arithmetic that the tests, the
smoke check and the benchmark's CPU-baseline leg compare the GPU library
against.  Shares no code with the GPU library; the GPU library never imports,
links or runs anything here.
"""
