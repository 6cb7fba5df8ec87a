"""MI355X (gfx950) SCR+AMG linear-solve library: see include/scr.h for the C ABI and
paper_2206_06996_amd.scr for its Python binding."""
