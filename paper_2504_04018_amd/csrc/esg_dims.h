// Vector dimensions for which search kernels are compiled.  One object file
// per entry is built from esg_search_inst.hip with -DESG_DIM=<d>.
#pragma once
#define ESG_DIMS(X) X(32) X(64) X(96) X(128) X(256) X(768)
