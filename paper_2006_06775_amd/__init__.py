"""MI355X (gfx950) hot path of the BioDynaMo agent engine: uniform-grid neighbour search,
sphere-sphere mechanics, spheroid growth/division and SIR epidemiology behind the C ABI of
libbdm.so (include/bdm.h).  ``bdm`` is the Python binding of that library."""
