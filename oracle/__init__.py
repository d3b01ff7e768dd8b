"""FP64 CPU oracle for the closed-loop virtual-trial path. Test infrastructure only."""
