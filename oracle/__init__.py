"""Plain, slow FP64 CPU oracle for the single-bit-upset injection path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  The device library never calls it, and it shares no code with the
HIP kernels or their host code: each function here is written from the paper's
definitions (or, where the paper is silent, from the documented reading of
3D Gaussian splatting) in float64 NumPy, in the order the method states.

Modules
    formats  storage formats, casts, bit flips            (Sec. 3; Lemma 1)
    guard    support box and clamp with counts            (Alg. 1; Thm. 1, Thm. 2)
    sh       real spherical-harmonic basis                (Sec. 3 "Parameter layout")
    render   activation, EWA projection, compositing      (Sec. 2 "Gaussian splatting"; Sec. 3)
    metrics  PSNR, footprint, catastrophe                 (Sec. 3 "Metrics"; Def. 1, Def. 2)
    scalar   pure-Python per-pixel renderer for tiny scenes, used only to pin `render`
"""
