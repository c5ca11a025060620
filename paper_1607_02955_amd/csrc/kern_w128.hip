// Kernel instantiations for block width 128.
#include "kern_impl.hpp"
CFC_DEFINE_TABLES(128)
