"""MI355X-native encrypted linear layers for hybrid FHE inference.

Submodules are imported explicitly:
  - ``fhelin``  : ctypes binding over the HIP library ``libfhelin.so``;
  - ``synth``   : seeded synthetic input generators (no scheme arithmetic);
  - ``serving`` : the continuous-batching request loop.
"""
