"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

Holds none of the method's arithmetic: it only produces propagator-shaped
random arrays and sink weights.  See ``synth.props`` for the definition.
"""
