"""Aggregate risk analysis on AMD Instinct MI355X (gfx950).

The engine implements the analysis stage of Bahl, Baltzer, Rau-Chaplin and
Varghese, "Parallel Simulations for Analysing Portfolios of Catastrophic Event
Risk" (Section II): Year Event Table + Event Loss Tables + layer terms in,
Year Loss Table + PML + TVaR out.  The computation lives in the HIP library
``libara.so`` behind the C-ABI of ``include/ara.h``; ``paper_1308_2066_amd.ara``
is its Python binding (same names) and ``paper_1308_2066_amd.session`` uploads
numpy inputs into handles.  Build with ``python -m paper_1308_2066_amd.build``.
"""
__all__ = ["ara", "session", "build"]
