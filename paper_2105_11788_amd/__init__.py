"""MI355X-native strong-bisimulation partition refinement (gfx950 HIP).

Submodules (imported explicitly, so that importing the package needs no GPU):
  bisim   binding of libbisim.so (include/bisim.h)
  gen     seeded synthetic LTS generators
  build   hipcc build of libbisim.so
"""
