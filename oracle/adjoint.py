"""Reverse sweep of the oracle step (discrete adjoint) -- not written yet."""
