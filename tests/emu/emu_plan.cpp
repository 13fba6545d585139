#include "../../paper_2606_28113_amd/csrc/plan.hip"
