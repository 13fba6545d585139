#include "../../paper_2606_28113_amd/csrc/kernels.hip"
