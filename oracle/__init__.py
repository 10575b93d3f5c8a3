"""CPU oracle for the self-adaptive Ising machine -- TEST INFRASTRUCTURE ONLY.

Plain, exact reference implementations used by tests/, the smoke check and the
bench's CPU baseline.  The product path never imports anything from here.
"""
