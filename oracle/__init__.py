"""Plain CPU oracle for the 16-point orthogonal approximate DCT (da Silveira,
Cintra, Bayer, Coelho, Kulasekera, Madanayake, Rajapaksha: "An Orthogonal
16-point Approximate DCT for Image and Video Compression").

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the
CPU-baseline leg of the benchmark may import this package.  The product path
(the HIP library and its Python binding) never imports, calls or links it,
and it shares no code, tables or helpers with that path.

Everything here is a direct, slow transcription of a definition in the paper
(or of the plain mathematics the paper relies on), computed with dense
matrices in int64 or float64.  No butterfly, blocking trick or fusion is
used; the fast factorisation of Eq. (1) appears only as matrices whose
product the tests compare with the literal T.

Modules
  transform  the matrices T, S, C_hat, the exact DCT-II and the Eq. (1)
             factors; blockwise forward and inverse transforms.
  codec      blocking of images, retention masks, the uniform quantiser,
             reconstruction rounding, SSE/PSNR, SSIM.
  metrics    the similarity and coding measures of Section 3 (Table 2).

Parity status: every function is pinned by a test against something the
paper prints or the mathematics fixes (see tests/test_oracle_pins.py), with
one exception noted in its docstring: ``codec.ssim`` follows the SSIM
definition the paper cites rather than anything the paper prints.
"""
from . import transform, codec, metrics  # noqa: F401
