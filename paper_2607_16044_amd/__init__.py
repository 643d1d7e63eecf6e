"""MI355X (gfx950) engine for the geometry-split ARK-IMEX scheme with explicit DG-IP and implicit
HDG-IP / HDG-MX (Ellmenreich, Shehadi, Lederer).  The numerical work runs in the HIP library
libimexhdg.so behind the C ABI of include/imexhdg.h; ``binding`` marshals torch tensors into it."""
