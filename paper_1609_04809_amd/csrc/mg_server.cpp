// serving scheduler (filled in below)
