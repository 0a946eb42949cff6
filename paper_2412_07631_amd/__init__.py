"""Direct algebraic CT reconstruction (factor A = QR once, X = R^-1 Q^T B) on
AMD Instinct MI355X (gfx950).

Submodules:
  ctqr  -- the binding to the HIP library ``libctqr.so`` (loads it on import
           and fails loudly if it is not built);
  synth -- seeded synthetic inputs (geometries, phantoms, noise).
"""
