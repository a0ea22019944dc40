"""CPU FP64 oracle for randomized Householder QR (Grigori & Timsit, arXiv 2405.10923).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, header, table
or constant generator with the HIP library; the two meet only through the
seeded input generators of ``paper_2405_10923_amd.inputs``.

Every routine is a plain, slow transcription of the paper's definitions and
algorithms in float64, written for checking by eye against the paper:

* ``philox``  -- counter-based generator used to draw the sketch (the paper
  leaves the generator unspecified; Philox4x64-10 is this project's choice).
* ``sketch``  -- the SRHT and Gaussian embeddings of Sec. 2.3, the structured
  sketch Psi of eq. (psi) and the sketching routine RHSketch (Alg. 1).
* ``rhqr``    -- RHVector (Alg. 2), right-looking RHQR (Alg. 3), left-looking
  RHQR (Alg. 4), deterministic Householder QR (Sec. 2.2), the thin Q factor
  (Sec. 3.2), recRHQR (Alg. 6) and its Randomized-Cholesky-QR variant.
* ``arnoldi`` -- RHQR-Arnoldi (Alg. 7) and RHQR-GMRES (Alg. 8).
* ``rgs``     -- BLAS2-RGS (Alg. 9) and plain randomized Gram-Schmidt.
* ``metrics`` -- factorization error, sketch orthogonality, condition numbers.
"""
