"""MI355X coagulation-fragmentation hot path: the C ABI of libcoag (coag.py),
its autograd wrapper (autograd.py) and the seeded synthetic discs (disc.py)."""
