"""CPU oracle of the scenario absorber interior-point method (float64).

TEST INFRASTRUCTURE ONLY: ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the product path never does.
It shares no code with the GPU path.
"""
