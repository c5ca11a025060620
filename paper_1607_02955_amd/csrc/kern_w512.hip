// Kernel instantiations for block width 512.
#include "kern_impl.hpp"
CFC_DEFINE_TABLES(512)
